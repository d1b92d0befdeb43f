"""Benchmark: FD-CGKS S2O4 steps on one MI355X.

Workload: 2D Navier-Stokes doubly periodic double shear layer, 2048 x 2048
primary + 2048 x 2048 dual nodes, Re = 1e4 (mu = 1e-4), Pr = 0.72,
gamma = 1.4, Ma = 0.15, tanh profile of thickness 1/80 with a seeded 5 %
sinusoidal perturbation, CFL 0.5 (time step reduced on the device every
step), FP64 throughout.  A step is two S2O4 stages, each a full pass of the
hot path (halo fill, interface sweep, node sweep, assemble + update) over
both grids.

Prints one JSON line.  value = node-updates per second per stage =
(N_primary + N_dual) * 2 stages * steps / seconds, inputs resident in HBM.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 2048
CFL = 0.5
MU, PR = 1e-4, 0.72
PEAK_FP64_TFLOPS = 78.6        # MI355X FP64 vector peak
PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
HBM_BYTES_PER_NODE_STAGE = 288  # algorithmic: stage 1 reads 12 / writes 24 doubles, stage 2 reads 24 / writes 12
# Dominant kernel of the default stage: k_fused2d<1,double,false>, the stage-1
# interface sweep fused with the update.  Unit of work: one node update (its
# share of the interface points, each two GENO line reconstructions, two
# gas-kinetic solves and the blend, plus the compact-flux assembly and the
# S2O4 update); one launch updates 2 n^2 nodes.  FP64 flops per node and HBM
# bytes per launch are from the rocprofv3 counters of this kernel
# (profiles/k_fused2d_shear2048.md: 64 x (ADD + MUL + 2 FMA + TRANS) wave
# instructions; FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000 after the copy-kernel
# calibration).  Both are None whenever the kernel has changed since the
# counters were taken.
FLOPS_PER_NODE_FUSED_STAGE1 = 6344
TRAFFIC_BYTES_PER_LAUNCH_FUSED_STAGE1 = 4.981e9
# With --separate: the stage-1 interface sweep k_edges2d<1,double,false>, unit
# one interface point, 2 (n+3)^2 per launch (profiles/k_edges2d_shear2048.md,
# same counters).
FLOPS_PER_IFACE_POINT_STAGE1 = 5618
TRAFFIC_BYTES_PER_LAUNCH_STAGE1 = 4.473e9
# 3D leg: the stage-1 interface sweep k_edges3d<true,false>, unit one solve
# (12 per cell), from profiles/k_edges3d_taylor_green128.md (same counters).
FLOPS_PER_SOLVE_3D_STAGE1 = 4797


# Launch shapes fdcgks_autotune picks on this workload (interface sweep,
# node sweep, update); fixed here so that profiled runs launch exactly what
# the timed run launches.
DEFAULT_TILES = "edge=64x2,node=64x1,update=128x1"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=N)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=N, help="side of the oracle's timed workload")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 1D periodic, 1D shock-tube and 512^2 vortex legs")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-per-problem comparison")
    ap.add_argument("--batch-steps", type=int, default=32)
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint-vs-forward comparison")
    ap.add_argument("--tiles", default=DEFAULT_TILES,
                    help="launch shapes kernel=XxY,... (default: the autotuner's pick at 2048^2)")
    ap.add_argument("--autotune", action="store_true", help="run fdcgks_autotune instead of --tiles")
    ap.add_argument("--separate", action="store_true",
                    help="run the separate interface sweep, node sweep and update (no fused stage kernel)")
    ap.add_argument("--no-graph", action="store_true", help="skip the small-problem graph-replay comparison")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-flux variant comparison")
    ap.add_argument("--no-char", action="store_true",
                    help="skip the characteristic-variable reconstruction comparison")
    ap.add_argument("--no-bounded", action="store_true", help="skip the walled-domain leg")
    ap.add_argument("--no-order8", action="store_true", help="skip the order-8 compact flux comparison")
    ap.add_argument("--no-pcie", action="store_true", help="skip the host-buffer (PCIe-inclusive) leg")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D (four-grid) leg")
    ap.add_argument("--n3d", type=int, default=128, help="side of the 3D Taylor-Green leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 512 MiB device copy first (reference for HBM byte counters)")
    return ap.parse_args()


def _host_info():
    """Threads the oracle may use, logical CPUs, and the CPU model of this host."""
    import ctypes
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    try:
        f = getattr(ctypes.CDLL(None), "omp_get_max_threads", None)
        if f:
            threads = int(f())
    except OSError:
        pass
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return threads, {"nproc": os.cpu_count(), "affinity_cpus": aff, "cpu_model": model}


def cpu_baseline(n):
    """The oracle, unmodified, timed on this host: stage 1 of one S2O4 step of
    the n x n workload itself (the full-size state; stage 2 does less work, so
    the per-stage rate is a bound from below), plus whole runs of the small
    configurations (1D periodic, 1D shock tubes) and one step of the 512^2
    vortex."""
    import workloads as WL
    from oracle import oracle as O
    threads, host = _host_info()
    pr = WL.shear_layer(n, seed=0, mu=MU, prandtl=PR)
    par = O.make_par(dim=2, nx=n, ny=n, lx=1.0, mu=MU, prandtl=PR)
    dt = O.dt2d(par, pr.P, pr.D, CFL)
    t0 = time.perf_counter()
    O.stage2d(par, 1, dt, pr.P, pr.D)
    sec = time.perf_counter() - t0
    del pr
    out = {"value": 2 * n * n / sec, "unit": "node-updates/s", "cores": threads, "kind": "oracle",
           "sample": f"stage 1 of one S2O4 step of the {n}x{n} double shear layer (the full-size state, "
                     f"{2 * n * n} nodes), {sec:.1f} s on {threads} threads", **host}
    cfg = {}
    # 1D periodic, N = 100 + shifted copy, to t = 2
    a = WL.advection1d(100, seed=0)
    p1 = O.make_par(dim=1, nx=100, lx=2.0, dual_1d=1)
    t0 = time.perf_counter()
    _, tt, k = O.step1d(p1, a.S, 100000, cfl=CFL, t_end=2.0)
    sec = time.perf_counter() - t0
    cfg["1d_periodic"] = {"steps": k, "t": tt, "seconds": round(sec, 3),
                          "node_updates_per_s": 2 * 100 * 2 * k / sec}
    # 1D shock tubes, N = 400, seeds 0..2, to t = 0.2
    tubes = []
    for seed in range(3):
        tb = WL.seeded_shock_tube(400, seed)
        p2 = O.make_par(dim=1, nx=400, lx=1.0, bc="zero_gradient")
        t0 = time.perf_counter()
        _, tt, k = O.step1d(p2, tb.S, 100000, cfl=CFL, t_end=0.2)
        sec = time.perf_counter() - t0
        tubes.append({"seed": seed, "steps": k, "seconds": round(sec, 3), "node_updates_per_s": 400 * 2 * k / sec})
    cfg["1d_shock_tubes"] = tubes
    # 2D vortex 512^2: one CFL step (a whole 10-step run is ten of these)
    v = WL.vortex(512, seed=0)
    p3 = O.make_par(dim=2, nx=512, ny=512, lx=v.lx)
    t0 = time.perf_counter()
    O.step2d(p3, v.P, v.D, 1, cfl=CFL)
    sec = time.perf_counter() - t0
    cfg["vortex_512"] = {"sample": "one CFL step", "seconds_per_step": round(sec, 3),
                         "node_updates_per_s": 2 * 512 * 512 * 2 / sec}
    # 3D Taylor-Green vortex: stage 1 at 32^3 (the GPU leg runs 128^3)
    tg = WL.taylor_green3d(32)
    p4 = O.make_par(dim=3, nx=32, ny=32, nz=32, lx=tg.lx, mu=tg.params["mu"], prandtl=PR)
    dt4 = O.dt3d(p4, tg.S, 0.4)
    t0 = time.perf_counter()
    O.stage3d(p4, 1, dt4, tg.S)
    sec = time.perf_counter() - t0
    cfg["taylor_green_3d"] = {"sample": "stage 1 of one step at 32^3 x 4 grids", "seconds": round(sec, 3),
                              "node_updates_per_s": 4 * 32 ** 3 / sec}
    out["configs"] = cfg
    return out


def config_legs(tiles):
    """The smaller configurations on the GPU: the 1D periodic run (N = 100 +
    shifted copy, noise seed 0, CFL 0.5 to t = 2), the seeded 1D shock tubes
    (N = 400, seeds 0..2, CFL 0.5 to t = 0.2; one launch per run), and the
    512^2 isentropic vortex (10 CFL steps, FP64 and the FP32-flux variant).
    Rates are node-updates per second per stage over the whole run, inputs
    resident on the device, first run untimed."""
    import torch

    import workloads as WL
    from paper_2606_17772_amd import Problem, make_params
    dev = torch.device("cuda:0")

    def run1d(prm, S, t_end):
        pb = Problem(prm)
        for g in range(S.shape[0]):
            pb.set_state_stacked(g, S[g])
        pb.step(nsteps=100000, cfl=CFL, t_end=t_end)  # warm-up run
        for g in range(S.shape[0]):
            pb.set_state_stacked(g, S[g])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tt, k = pb.step(nsteps=100000, cfl=CFL, t_end=t_end)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, tt, k

    out = {}
    a = WL.advection1d(100, seed=0)
    sec, tt, k = run1d(make_params(dim=1, nx=100, lx=2.0, dual_1d=1), a.S, 2.0)
    out["1d_periodic"] = {"workload": "1D Euler, periodic [0,2], N=100 + 100 shifted, noise seed 0, CFL 0.5 to t=2",
                          "steps": k, "t": tt, "ms": round(sec * 1e3, 3), "node_updates_per_s": 2 * 100 * 2 * k / sec}
    tubes = []
    for seed in range(3):
        tb = WL.seeded_shock_tube(400, seed)
        sec, tt, k = run1d(make_params(dim=1, nx=400, lx=1.0, bc="zero_gradient"), tb.S, 0.2)
        tubes.append({"seed": seed, "left": tb.params["left"], "right": tb.params["right"], "steps": k,
                      "ms": round(sec * 1e3, 3), "node_updates_per_s": 400 * 2 * k / sec})
    out["1d_shock_tubes"] = {"workload": "1D Euler shock tubes, N=400 on [0,1], seeded states, zero-gradient ends, "
                                         "CFL 0.5 to t=0.2", "runs": tubes}
    v = WL.vortex(512, seed=0)
    S0 = torch.from_numpy(np.stack([v.P, v.D])).to(dev)
    res = {}
    for name, kw in (("fp64", {}), ("fp32_flux", {"fp32_flux": True})):
        pb = Problem(make_params(dim=2, nx=512, ny=512, lx=v.lx, ly=v.ly, **kw))
        for tname, (x, y) in tiles.items():
            pb.set_tile(tname, x, y)
        pb.set_state_all(S0)
        pb.step(nsteps=10, cfl=CFL)
        pb.set_state_all(S0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, k = pb.step(nsteps=10, cfl=CFL)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        res[name] = (sec, k, pb.get_state_all(device=dev))
        del pb
    (s64, k64, S64), (s32, k32, S32) = res["fp64"], res["fp32_flux"]
    out["vortex_512"] = {"workload": "2D Euler isentropic vortex, periodic [0,10]^2, 512^2 + dual, beta 5, seed 0, "
                                     "10 CFL-0.5 steps", "steps": k64, "fp64_ms_per_step": round(s64 / k64 * 1e3, 4),
                         "fp64_node_updates_per_s": 2 * 512 * 512 * 2 * k64 / s64,
                         "fp32_flux_ms_per_step": round(s32 / k32 * 1e3, 4),
                         "fp32_flux_node_updates_per_s": 2 * 512 * 512 * 2 * k32 / s32,
                         "fp32_flux_max_rel_diff_values_vs_fp64": _max_rel_values(S64, S32)}
    return out


BATCH_CFL = 0.4  # the four-quadrant Riemann members need CFL <= 0.4 (the paper's tests use CFL >= 0.4)


def batch_comparison(steps):
    """64 independent 2D Euler problems (sides seeded in [64, 512]; vortex
    members periodic, four-quadrant Riemann members with zero-gradient sides,
    CFL 0.4) advanced by the batched launches (one launch per phase captured
    as HIP graphs of 16 steps; the same launches uncaptured; one cooperative
    persistent launch per stage) and by a loop over single problems (each
    with its own captured step graphs) on the same GPU."""
    import torch

    import workloads as WL
    from paper_2606_17772_amd import Batch, Problem, make_params
    probs = WL.batch_problems(64, 64, 512, seed=0, bounded=True)
    prms = [make_params(dim=2, nx=p.nx, ny=p.ny, lx=p.lx, ly=p.ly, bc=p.params.get("bc", "periodic"))
            for p in probs]
    bounded = [p.params.get("bc", "periodic") != "periodic" for p in probs]
    nodes = sum(p.nx * p.ny + (p.nx + b) * (p.ny + b) for p, b in zip(probs, bounded))
    out = {"members": len(probs), "zero_gradient_members": int(sum(bounded)), "nodes_per_stage": nodes,
           "steps": steps}
    rates, states = {}, {}
    for mode in ("graph", "phased", "persistent"):
        B = Batch(prms)
        B.set_mode(mode)
        for m, p in enumerate(probs):
            B.set_state_stacked(m, 0, p.P)
            B.set_state_stacked(m, 1, p.D)
        B.step(nsteps=1, cfl=BATCH_CFL)
        B.step(nsteps=16, cfl=BATCH_CFL)  # captures the graphs (graph mode)
        for m, p in enumerate(probs):
            B.set_state_stacked(m, 0, p.P)
            B.set_state_stacked(m, 1, p.D)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.step(nsteps=steps, cfl=BATCH_CFL)
        torch.cuda.synchronize()
        rates[mode] = nodes * 2 * steps / (time.perf_counter() - t0)
        states[mode] = [B.get_state_stacked(m, 0) for m in (0, 1, 63)]
        del B
    singles = [Problem(q) for q in prms]
    for m, p in enumerate(probs):
        singles[m].set_state_stacked(0, p.P)
        singles[m].set_state_stacked(1, p.D)
    for pb in singles:
        pb.step(nsteps=16, cfl=BATCH_CFL)  # captures each problem's step graphs
    for m, p in enumerate(probs):
        singles[m].set_state_stacked(0, p.P)
        singles[m].set_state_stacked(1, p.D)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pb in singles:
        pb.step(nsteps=steps, cfl=BATCH_CFL)
    torch.cuda.synchronize()
    loop = nodes * 2 * steps / (time.perf_counter() - t0)
    same = all(np.array_equal(states[md][q], singles[m].get_state_stacked(0))
               for md in states for q, m in enumerate((0, 1, 63)))
    out.update({"graph_node_updates_per_s": rates["graph"], "phased_node_updates_per_s": rates["phased"],
                "persistent_node_updates_per_s": rates["persistent"],
                "per_problem_loop_node_updates_per_s": loop,
                "speedup_graph": rates["graph"] / loop, "speedup_phased": rates["phased"] / loop,
                "speedup_persistent": rates["persistent"] / loop,
                "bitwise_equal_sampled_members": bool(same)})
    return out


def _variant_runs(pr, n, tiles, variants, steps):
    """Time `steps` steps of the workload for each keyword set in `variants`
    (all at the first variant's CFL dt, from the same resident state):
    [(ms per step, final state, per-kernel ms per step)]."""
    import torch

    from paper_2606_17772_amd import Problem, make_params
    dev = torch.device("cuda:0")
    S0 = torch.from_numpy(np.stack([pr.P, pr.D])).to(dev)
    out, dt = [], None
    for kw in variants:
        pb = Problem(make_params(dim=2, nx=n, ny=n, lx=1.0, ly=1.0, mu=MU, prandtl=PR, **kw))
        for name, (x, y) in tiles.items():
            pb.set_tile(name, x, y)
        pb.set_state_all(S0)
        if dt is None:
            dt = pb.compute_dt(CFL)
        pb.step(nsteps=2, dt=dt)
        pb.set_state_all(S0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pb.step(nsteps=steps, dt=dt)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        S = pb.get_state_all(device=dev)
        pb.set_state_all(S0)
        _, _, kms = pb.step_timed(nsteps=2, dt=dt)
        out.append((ms, S, {k: round(v / 2, 4) for k, v in kms.items()}))
        del pb
    return out


def _max_rel_values(a, b):
    a, b = a[:, :4], b[:, :4]
    return float(((a - b).abs().amax(dim=(2, 3)) / a.abs().amax(dim=(2, 3))).max())


def fp32_flux_comparison(pr, n, tiles, steps=10):
    """The FP32-flux variant (gas-kinetic solvers in FP32, reconstruction,
    assembly and update in FP64) on the same workload: time per step and the
    largest relative difference of the values W from the FP64 path after
    the same number of steps (per plane, relative to the plane's largest
    value)."""
    (m64, S64, _), (m32, S32, _) = _variant_runs(pr, n, tiles, [{}, {"fp32_flux": True}], steps)
    return {"workload": f"{n}x{n} shear layer, {steps} steps at the FP64 path's CFL dt",
            "fp64_ms_per_step": round(m64, 3), "fp32_flux_ms_per_step": round(m32, 3),
            "speedup": round(m64 / m32, 3), "max_rel_diff_values_vs_fp64": _max_rel_values(S64, S32)}


def characteristic_comparison(pr, n, tiles, steps=10):
    """Reconstruction in characteristic variables (Sec. 3) on the same
    workload: node-update rate, time per step and per kernel, and the largest
    relative difference of the values W from the conservative-variable path
    after the same steps (a scheme difference, not round-off)."""
    runs = _variant_runs(pr, n, tiles, [{}, {"recon_vars": "characteristic"}], steps)
    (mc, Sc, kc), (mh, Sh, kh) = runs
    nodes = 2 * n * n
    return {"workload": f"{n}x{n} shear layer, {steps} steps at the conservative path's CFL dt",
            "node_updates_per_s": nodes * 2 / (mh * 1e-3), "ms_per_step": round(mh, 3),
            "conservative_ms_per_step": round(mc, 3), "slowdown_vs_conservative": round(mh / mc, 3),
            "kernel_ms_per_step": kh, "conservative_kernel_ms_per_step": kc,
            "max_rel_diff_values_vs_conservative": _max_rel_values(Sc, Sh)}


def pcie_inclusive(pb, pr, n, steps):
    """The boundary's host path: both grids' state handed over from host
    (pageable numpy) arrays, `steps` CFL steps, and the state read back into
    host arrays.  Node-update rate including both transfers, and the transfer
    times; `value` excludes them (inputs already resident in HBM)."""
    import torch
    t0 = time.perf_counter()
    for g, S in ((0, pr.P), (1, pr.D)):
        pb.set_state(g, S[0:4], S[4:8], S[8:12])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, k = pb.step(nsteps=steps, cfl=CFL)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out = [pb.get_state(g) for g in (0, 1)]
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    assert k == steps and out[1][0].shape == (4, n, n)
    nbytes = 2 * pr.P.nbytes
    return {"workload": f"{n}x{n} shear layer: state in from host arrays, {steps} CFL steps, state out to host arrays",
            "node_updates_per_s": 2 * n * n * 2 * steps / (t3 - t0), "host_to_device_ms": round((t1 - t0) * 1e3, 2),
            "steps_ms": round((t2 - t1) * 1e3, 2), "device_to_host_ms": round((t3 - t2) * 1e3, 2),
            "bytes_each_way": nbytes}


def order8_comparison(pr, n, tiles, steps=10):
    """The compact flux of order 8 (the wider stencil, nodal fluxes at
    j-1..j+2) on the same workload: node-update rate, time per step and per
    kernel against the order-6 flux, and the largest relative difference of
    the values W after the same steps (a discretisation difference)."""
    runs = _variant_runs(pr, n, tiles, [{}, {"flux_order": 8}], steps)
    (m6, S6, k6), (m8, S8, k8) = runs
    nodes = 2 * n * n
    return {"workload": f"{n}x{n} shear layer, {steps} steps at the order-6 path's CFL dt",
            "node_updates_per_s": nodes * 2 / (m8 * 1e-3), "ms_per_step": round(m8, 3),
            "order6_ms_per_step": round(m6, 3), "slowdown_vs_order6": round(m8 / m6, 3),
            "kernel_ms_per_step": k8, "order6_kernel_ms_per_step": k6,
            "max_rel_diff_values_vs_order6": _max_rel_values(S6, S8)}


def bounded_comparison(n, tiles, steps=10):
    """Bounded sides (walls) on a workload of the same size: a smooth flow
    in [0,1]^2 with adiabatic no-slip walls at x = 0, 1 and reflecting
    (symmetry) walls at y = 0, 1, Navier-Stokes at the shear layer's mu and
    Pr; the dual grid then has (n+1)^2 nodes.  Node-update rate and time
    per step against the periodic shear layer."""
    import torch

    import workloads as WL
    from paper_2606_17772_amd import Problem, make_params
    P, D = WL.sample_bounded(WL.mirror_flow(1.0, 1.0, 1, 1), n, n, 1.0 / n, 1, 1)
    pb = Problem(make_params(dim=2, nx=n, ny=n, lx=1.0, ly=1.0, mu=MU, prandtl=PR,
                             sides=("no_slip", "no_slip", "reflecting", "reflecting")))
    for name, (x, y) in tiles.items():
        pb.set_tile(name, x, y)
    pb.set_state_stacked(0, P)
    pb.set_state_stacked(1, D)
    pb.step(nsteps=2, cfl=CFL)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pb.step(nsteps=steps, cfl=CFL)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    nodes = n * n + (n + 1) * (n + 1)
    return {"workload": f"{n}x{n} (+ {n + 1}x{n + 1} dual) smooth flow, no-slip x walls, reflecting y walls, "
                        f"{steps} CFL steps", "ms_per_step": round(ms, 3),
            "node_updates_per_s": nodes * 2 / (ms * 1e-3)}


ADJ_STEPS, ADJ_EVERY, ADJ_CFL = 50, 7, 0.25


def adjoint_batch_gradient(count=64):
    """Gradient workload of the batched configuration: 64 members (sides
    seeded in [64, 512]; periodic vortices and four-quadrant Riemann
    problems with zero-gradient sides), each
    advanced 50 steps at a time step frozen from its initial state (CFL 0.25;
    a member whose frozen step goes non-physical is skipped and counted);
    J = 1/2 sum over members and primary nodes of (rho(T) - rho_target)^2 h^2,
    the target being the same run from the member's data drawn with another
    seed; the control is an additive density perturbation on the primary
    nodes (gradient = adjoint of the initial primary density).  Rollouts keep
    every 7th state and recompute the rest.  Timed against the plain forward
    steps of the same members, plus central-difference checks of the
    gradient of a vortex and a Riemann member along 8 random directions."""
    import torch

    import workloads as WL
    from paper_2606_17772_amd import FdcgksError, Problem, make_params
    from paper_2606_17772_amd.adjoint import density, get_state_vector, rollout, set_state_vector
    dev = torch.device("cuda:0")
    skipped = []
    sizes = WL.batch_sizes(count, 64, 512, seed=0)
    gen = lambda b, n, sd: WL.vortex(n, seed=sd) if b % 2 == 0 else WL.riemann2d_bounded(n, seed=sd)  # noqa: E731

    def state(pb, pr):  # the member's data in the rollout's state form (flat when the grids differ in size)
        if any(pb.bounded):
            return torch.from_numpy(np.concatenate([pr.P.ravel(), pr.D.ravel()])).to(dev)
        return torch.from_numpy(np.stack([pr.P, pr.D])).to(dev)
    t_fwd = t_grad = 0.0
    J_total, gnorm2, members = 0.0, [0.0, 0.0], 0
    checks = []
    for b, n in enumerate(sizes):
        pr, tg = gen(b, n, b), gen(b, n, 5000 + b)
        pb = Problem(make_params(dim=2, nx=n, ny=n, lx=pr.lx, ly=pr.ly, bc=pr.params.get("bc", "periodic")))
        S0 = state(pb, pr)
        set_state_vector(pb, S0)
        dt = pb.compute_dt(ADJ_CFL)
        try:
            for S in (state(pb, tg), S0):
                set_state_vector(pb, S)
                pb.step(nsteps=ADJ_STEPS, dt=dt)
        except FdcgksError:
            skipped.append(b)
            del pb
            continue
        set_state_vector(pb, state(pb, tg))
        pb.step(nsteps=ADJ_STEPS, dt=dt)
        rho_t = density(pb, get_state_vector(pb, dev)).clone()
        h2 = pr.h * pr.h
        # plain forward
        set_state_vector(pb, S0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pb.step(nsteps=ADJ_STEPS, dt=dt)
        torch.cuda.synchronize()
        t_fwd += time.perf_counter() - t0
        # gradient: checkpointed rollout + reverse sweep
        X = S0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = rollout(pb, X, dt, ADJ_STEPS, checkpoint_every=ADJ_EVERY)
        J = 0.5 * ((density(pb, out) - rho_t) ** 2).sum() * h2
        J.backward()
        grad = density(pb, X.grad)
        torch.cuda.synchronize()
        t_grad += time.perf_counter() - t0
        J_total += float(J.detach())
        gnorm2[b % 2] += float((grad * grad).sum())
        members += 1
        if b in (0, 1):  # central differences along 8 random density directions (vortex b = 0, Riemann b = 1)
            checks.append(_fd_directions(pb, S0, dt, rho_t, h2, grad, n, b))
        del pb, X, out, J
    return {"workload": f"{members} members (vortices periodic, Riemann problems with zero-gradient sides), sides in "
                        f"[64, 512], {ADJ_STEPS} steps at frozen CFL-{ADJ_CFL} dt, checkpoint every {ADJ_EVERY} steps",
            "skipped_nonphysical_members": skipped,
            "forward_s": round(t_fwd, 3), "gradient_s": round(t_grad, 3), "gradient_over_forward": round(t_grad / t_fwd, 2),
            "J": J_total, "grad_norm_vortex_members": gnorm2[0] ** 0.5, "fd_checks": checks}


def _fd_directions(pb, S0, dt, rho_t, h2, grad, n, b, ndir=8):
    """Adjoint directional derivatives <grad J, v> against central
    differences of J along `ndir` seeded random density directions v, at
    eps = 1e-6 and 1e-4 of the density scale.  On Riemann data the central
    difference itself depends on eps: J of the discrete scheme is not smooth
    at round-off level there (GENO's path function switches where smoothness
    indicators are ~0), so the adjoint is the derivative of a branch that a
    finite step leaves; such members are reported, not asserted."""
    import torch

    from paper_2606_17772_amd.adjoint import density, get_state_vector, set_state_vector
    dev = S0.device
    gen = torch.Generator(device=dev).manual_seed(100 + b)

    def Jof(v, e):
        S = S0.clone()
        density(pb, S).add_(e * v)
        set_state_vector(pb, S)
        pb.step(nsteps=ADJ_STEPS, dt=dt)
        return 0.5 * float(((density(pb, get_state_vector(pb, dev)) - rho_t) ** 2).sum()) * h2

    rel = {"1e-6": [], "1e-4": []}
    an_all, fd_all = [], []
    scale = float(density(pb, S0).abs().max())
    for _ in range(ndir):
        v = torch.randn(grad.shape, dtype=torch.float64, device=dev, generator=gen)
        v /= float(v.abs().max())
        an = float((grad * v).sum())
        an_all.append(an)
        for tag, f in (("1e-6", 1e-6), ("1e-4", 1e-4)):
            e = f * scale
            fd = (Jof(v, e) - Jof(v, -e)) / (2 * e)
            if tag == "1e-6":
                fd_all.append(fd)
            rel[tag].append(abs(an - fd) / max(abs(fd), 1e-300))
    kind = "vortex" if b % 2 == 0 else "riemann"
    worst = max(abs(a - f) for a, f in zip(an_all, fd_all)) / max(abs(f) for f in fd_all)
    out = {"member": b, "kind": kind, "side": n, "directions": ndir, "adjoint": an_all, "central_difference_1e-6": fd_all,
           "max_abs_diff_over_max_abs_fd_1e-6": worst,
           "max_rel_diff_eps_1e-6": max(rel["1e-6"]), "max_rel_diff_eps_1e-4": max(rel["1e-4"])}
    if kind == "riemann":
        out["note"] = ("J is not smooth at round-off level on piecewise-constant data (GENO path functions switch where "
                       "smoothness indicators vanish): compare the spread between the two eps")
    return out


def graph_comparison(n=64, steps=400):
    """Launch overhead: a small problem (n^2 isentropic vortex) stepped with
    the captured-step graphs (16 steps per graph) and with separate kernel
    launches."""
    import torch

    import workloads as WL
    from paper_2606_17772_amd import Problem, make_params
    pr = WL.vortex(n, seed=0)
    res = {}
    for mode in (True, False):
        pb = Problem(make_params(dim=2, nx=n, ny=n, lx=10.0, ly=10.0))
        pb.set_state_all(np.ascontiguousarray(np.stack([pr.P, pr.D])))
        pb.graph_steps = 16 if mode else 0
        pb.step(nsteps=16, cfl=CFL)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pb.step(nsteps=steps, cfl=CFL)
        torch.cuda.synchronize()
        res["graph" if mode else "separate"] = 2 * n * n * 2 * steps / (time.perf_counter() - t0)
        del pb
    return {"workload": f"{n}x{n} isentropic vortex, {steps} steps", "graph_node_updates_per_s": res["graph"],
            "separate_launch_node_updates_per_s": res["separate"], "speedup": res["graph"] / res["separate"]}


def three_d_leg(n=128, steps=5):
    """The 3D extension (four grids: primary plus the three face-offset
    duals): a Taylor-Green vortex, Re 1600, Ma 0.1, Pr 0.72, on n^3 cells per
    grid, stepped at a fixed CFL-0.4 dt; node-updates count all four grids.
    Not one of the paper's configurations (its tests are 1D and 2D)."""
    import torch

    import workloads as WL
    from paper_2606_17772_amd import Problem3D
    pr = WL.taylor_green3d(n)
    pb = Problem3D(nx=n, ny=n, nz=n, lx=pr.lx, mu=pr.params["mu"], prandtl=PR)
    dev = torch.device("cuda:0")
    for g in range(4):
        pb.set_state(g, torch.from_numpy(pr.S[g]).to(dev))
    dt = pb.compute_dt(0.4)
    pb.step(nsteps=1, dt=dt)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    _, k = pb.step(nsteps=steps, dt=dt)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    _, _, kms = pb.step_timed(nsteps=2, dt=dt)
    d = pb.diagnostics()
    nodes = 4 * n ** 3
    solves = 12 * n ** 3
    edge1 = kms["edge1"] / 2
    del pb
    torch.cuda.empty_cache()
    achieved = FLOPS_PER_SOLVE_3D_STAGE1 * solves / (edge1 * 1e-3) / 1e12
    return {"workload": f"3D Taylor-Green vortex {n}^3 x 4 grids, Re 1600, Ma 0.1, Pr 0.72, (6-4) GENO, FP64, "
                        f"fixed dt (CFL 0.4), {steps} steps",
            "node_updates_per_s": nodes * 2 / (ms * 1e-3), "ms_per_step": round(ms, 3),
            "kernel_ms_per_step": {k2: round(v / 2, 4) for k2, v in kms.items()},
            "interface_solves_per_s_stage1": solves / (edge1 * 1e-3),
            "roofline": {"kernel": "k_edges3d<true,false> (stage-1 interface sweep)", "bound": "alu",
                         "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "flop_per_solve": FLOPS_PER_SOLVE_3D_STAGE1,
                         "avg_launch_ms": round(edge1, 4)},
            "min_rho": d[20], "min_p": d[21]}


def adjoint_comparison(pb, n, reps=2):
    """Vector-Jacobian product of one step (fdcgks_step_vjp: forward
    recompute at the frozen dt, then the reverse sweep) on the same workload
    and state, against the forward step at the same dt.  Also the adjoint of
    the conserved dual-grid energy sum, whose exact value is the indicator
    itself (deviation = round-off of the periodic cancellation)."""
    import torch
    dev = torch.device("cuda:0")
    S = pb.get_state_all(device=dev)
    dt = pb.compute_dt(CFL)
    gen = torch.Generator(device=dev).manual_seed(0)
    lam = torch.randn(S.shape, dtype=torch.float64, device=dev, generator=gen)
    pb.step_vjp(dt, lam)  # first call allocates the adjoint workspace
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        pb.step_vjp(dt, lam)
    e1.record(stream)
    torch.cuda.synchronize()
    vjp_ms = e0.elapsed_time(e1) / reps
    e0.record(stream)
    pb.step(nsteps=reps, dt=dt)
    e1.record(stream)
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / reps
    pb.set_state_all(S)
    ind = torch.zeros_like(S)
    ind[1, 3] = 1.0
    dev_ind = float((pb.step_vjp(dt, ind) - ind).abs().max())
    return {"workload": f"one step of the {n}x{n} shear layer at its CFL dt, random adjoint seed",
            "vjp_ms": round(vjp_ms, 3), "forward_step_ms": round(fwd_ms, 3),
            "vjp_over_forward": round(vjp_ms / fwd_ms, 2),
            "conserved_sum_adjoint_max_deviation": dev_ind}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU decomposition is a design, not built", file=sys.stderr)
        sys.exit(2)
    import torch

    import workloads as WL
    from paper_2606_17772_amd import Problem, make_params

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.empty(64 * 2 ** 20, dtype=torch.float64, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    n = args.n
    pr = WL.shear_layer(n, seed=0, mu=MU, prandtl=PR)
    prm = make_params(dim=2, nx=n, ny=n, lx=1.0, ly=1.0, mu=MU, prandtl=PR)
    pb = Problem(prm)
    if args.separate:
        pb.fuse_stage = False  # otherwise the default: the fused stage kernel at this size
    dev = torch.device("cuda:0")
    # inputs resident in HBM before timing
    for g, S in ((0, pr.P), (1, pr.D)):
        T = torch.from_numpy(S).to(dev)
        pb.set_state(g, T[0:4].contiguous(), T[4:8].contiguous(), T[8:12].contiguous())
    torch.cuda.synchronize()
    if args.autotune:
        tiles = pb.autotune(reps=5)
    else:
        for item in args.tiles.split(","):
            name, xy = item.split("=")
            x, y = (int(v) for v in xy.split("x"))
            pb.set_tile(name, x, y)
        tiles = pb.tiles()
    t = 0.0
    if args.warmup:
        t, _ = pb.step(nsteps=args.warmup, cfl=CFL, t=t)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t, k = pb.step(nsteps=args.steps, cfl=CFL, t=t)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    assert k == args.steps
    nodes = 2 * n * n
    value = nodes * 2 * args.steps / (ms * 1e-3)
    # per-kernel breakdown on the same stream (separate, untimed-for-value run)
    _, _, kms = pb.step_timed(nsteps=max(2, args.steps // 4), cfl=CFL, t=t)
    kn = max(2, args.steps // 4)
    fused = kms["edge1"] == 0.0  # no separate interface sweep ran
    if fused:
        # the fused kernel's launches are timed under the update slot
        launch_ms = kms["update1"] / kn
        flops_per_unit, units, traffic = FLOPS_PER_NODE_FUSED_STAGE1, 2 * n * n, TRAFFIC_BYTES_PER_LAUNCH_FUSED_STAGE1
        kernel = "k_fused2d<1,double,false> (stage-1 interface sweep fused with the update)"
    else:
        launch_ms = kms["edge1"] / kn
        flops_per_unit, units, traffic = FLOPS_PER_IFACE_POINT_STAGE1, 2 * (n + 3) * (n + 3), \
            TRAFFIC_BYTES_PER_LAUNCH_STAGE1
        kernel = "k_edges2d<1,double,false> (stage-1 interface sweep)"
    if flops_per_unit:
        achieved = flops_per_unit * units / (launch_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": traffic}
    else:
        roof = {"bound": "alu", "achieved": None, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": None,
                "traffic": None}
    roof["kernel"] = kernel
    roof["avg_launch_ms"] = round(launch_ms, 4)
    hbm_gbs = value * HBM_BYTES_PER_NODE_STAGE / 1e9
    out = {
        "metric": "node-updates/s per stage (FP64, 1 GPU)",
        "value": value,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"2D Navier-Stokes double shear layer {n}x{n} primary + dual, Re=1e4, Pr=0.72, "
                               "CFL 0.5, (6-4) GENO, FP64", "nodes_per_stage": nodes, "stages_per_step": 2,
                   "launch_shapes": {k2: f"{x}x{y}" for k2, (x, y) in tiles.items()}, "step_graphs": True,
                   "stage": "fused" if fused else "separate"},
        "roofline": roof,
        "hbm_roofline": {"algorithmic_bytes_per_node_stage": HBM_BYTES_PER_NODE_STAGE,
                         "achieved_GBs": round(hbm_gbs, 1), "peak_GBs": PEAK_HBM_GBS,
                         "frac": round(hbm_gbs / PEAK_HBM_GBS, 4)},
        "kernel_ms_per_step": {k2: round(v / kn, 4) for k2, v in kms.items()},
    }
    if not args.no_pcie:
        out["pcie_inclusive"] = pcie_inclusive(pb, pr, n, args.steps)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_comparison(pb, n)
    if not args.no_fp32 or not args.no_char or not args.no_bounded or not args.no_order8:
        del pb
        torch.cuda.empty_cache()
        pb = None
    if not args.no_fp32:
        out["fp32_flux"] = fp32_flux_comparison(pr, n, tiles)
    if not args.no_char:
        out["characteristic"] = characteristic_comparison(pr, n, tiles)
    if not args.no_order8:
        out["order8"] = order8_comparison(pr, n, tiles)
    if not args.no_bounded:
        torch.cuda.empty_cache()
        out["bounded"] = bounded_comparison(n, tiles)
    if not args.no_graph:
        out["graph_replay"] = graph_comparison()
    if not args.no_3d:
        torch.cuda.empty_cache()
        out["three_d"] = three_d_leg(args.n3d)
    if not args.no_configs:
        out["configs"] = config_legs(tiles)
    if not args.no_batch:
        del pb
        torch.cuda.empty_cache()
        out["batched"] = batch_comparison(args.batch_steps)
    if not args.no_adjoint and not args.no_batch:
        torch.cuda.empty_cache()
        out["batched_adjoint_gradient"] = adjoint_batch_gradient()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
