"""Parity of the order-8 compact flux (flux_order = 8: the wider stencil of
Sec. 2.1, the averaging conditions also on the nodal cells j-1 and j+2)
against the oracle (GPU).

Stages element by element at the 1e-12 bar on periodic and walled 2D
problems and on 1D lines; CFL steps against max(1e-12, 4 x the oracle's
one-ulp sensitivity); the order of accuracy measured through the GPU path
on the smooth 1D advection test (it must exceed 7, against about 6 with the
order-6 flux); the graph and fused-node options.  Batches and the step
adjoint with this flux: test_gpu_batch.py, test_gpu_adjoint.py."""
import numpy as np
import pytest

import workloads as WL
from tests import test_gpu_boundaries as TB
from tests import test_gpu_parity1d as T1
from tests.helpers import (TOL, check_full_size_sampled, floors_state, gpu_params, oracle_par, ref_scales, relerr,
                           settings, ulp_sensitivity)

pytestmark = pytest.mark.gpu


def _w8(case):
    s, P, D = case
    return dict(s, flux_order=8), P, D


def _periodic(s, pr):
    return dict(s, flux_order=8), pr.P, pr.D


CASES = {
    "rough_67x9": lambda: _periodic(settings(dim=2, nx=67, ny=9, lx=1.0), WL.random_rough2d(67, 9, seed=8)),
    "riemann_33_62": lambda: _periodic(settings(dim=2, nx=33, ny=33, lx=1.0, variant="6-2"),
                                       WL.riemann2d(33, seed=9)),
    "vortex_40_linear": lambda: _periodic(settings(dim=2, nx=40, ny=40, lx=10.0, variant="linear"),
                                          WL.vortex(40, seed=2)),
    "shear_ns_36": lambda: _periodic(settings(dim=2, nx=36, ny=36, lx=1.0, mu=1e-3, prandtl=0.72),
                                     WL.shear_layer(36, seed=3, k=20.0)),
    "mixed_48x20": lambda: _w8(TB._case_mixed()),
    "zero_gradient_riemann_33": lambda: _w8(TB._case_zerograd_riemann()),
    "no_slip_ns_40x8": lambda: _w8(TB._case_noslip_ns()),
    "reflecting_all_char_67x9": lambda: _w8(TB._case_refl_all(recon_vars="characteristic")),
}


def _problem(s, P, D):
    from paper_2606_17772_amd import Problem
    pb = Problem(gpu_params(s))
    pb.set_state_stacked(0, P)
    pb.set_state_stacked(1, D)
    return pb


def _floors(s, P, D):
    return floors_state(ref_scales([P, D], s["gamma"], s["lx"]))


@pytest.mark.parametrize("name", list(CASES))
def test_stages_order8(oracle, name):
    s, P, D = CASES[name]()
    print(f"order-8 stages: {name}", flush=True)
    dt = 0.2 * (s["lx"] / s["nx"]) / 3.0
    par = oracle_par(oracle, s)
    oP, oD, aP, aD = oracle.stage2d(par, 1, dt, P, D)
    o2P, o2D = oracle.stage2d(par, 2, dt, oP, oD, aP, aD)
    pb = _problem(s, P, D)
    fl = _floors(s, P, D)
    g1, ga = pb.debug_stage(1, dt)
    for g, o in ((g1[0], oP), (g1[1], oD), (ga[0], aP), (ga[1], aD)):
        err, where = relerr(g, o, fl)
        assert err <= TOL, (where, err)
    g2 = pb.debug_stage(2, dt)
    for g, o in ((g2[0], o2P), (g2[1], o2D)):
        err, where = relerr(g, o, fl)
        assert err <= TOL, (where, err)
    # the order-6 flux gives a different stage: the wider stencil is in use
    s6 = dict(s, flux_order=6)
    o6P = oracle.stage2d(oracle_par(oracle, s6), 1, dt, P, D)[0]
    assert relerr(o6P, oP, fl)[0] > 100 * TOL


@pytest.mark.parametrize("name,nsteps", [("shear_ns_36", 3), ("mixed_48x20", 3), ("riemann_33_62", 2)])
def test_steps_order8(oracle, name, nsteps):
    s, P, D = CASES[name]()
    par = oracle_par(oracle, s)
    pb = _problem(s, P, D)
    oP, oD, ot, ok = oracle.step2d(par, P, D, nsteps, cfl=0.5)
    t, n = pb.step(nsteps=nsteps, cfl=0.5)
    assert n == nsteps == ok and abs(t - ot) <= 1e-13 * ot
    fl = _floors(s, P, D)
    sens = ulp_sensitivity(lambda A, B: oracle.step2d(par, A, B, nsteps, cfl=0.5)[:2], P, D, fl)
    for g, o in ((pb.get_state_stacked(0), oP), (pb.get_state_stacked(1), oD)):
        err, where = relerr(g, o, fl)
        print(f"order 8, {name}, {nsteps} steps: gpu-oracle {err:.2e}, oracle 1-ulp sensitivity {sens:.2e}")
        assert err <= max(TOL, 4 * sens), (where, err, sens)


@pytest.mark.parametrize("name", ["shear_ns_36", "mixed_48x20"])
def test_graph_and_fused_option_order8(name):
    """Captured steps equal eager ones bit for bit; the fused node option
    (whose tile holds a one-node halo) falls back to the separate kernels."""
    s, P, D = CASES[name]()
    a = _problem(s, P, D)
    a.use_graph = False
    a.step(nsteps=5, cfl=0.5)
    b = _problem(s, P, D)
    b.graph_steps = 4
    b.fuse_nodes = True
    b.step(nsteps=5, cfl=0.5)
    for g in (0, 1):
        assert np.array_equal(a.get_state_stacked(g), b.get_state_stacked(g))


def test_full_size_sampled_order8(oracle):
    """The order-8 flux on the 2048^2 shear layer (the benchmark's order-8
    leg): both stages on sampled nodes (bars: check_full_size_sampled)."""
    n = 2048
    pr = WL.shear_layer(n, seed=0)
    s = settings(dim=2, nx=n, ny=n, lx=1.0, mu=1e-4, prandtl=0.72, flux_order=8)
    pb = _problem(s, pr.P, pr.D)
    check_full_size_sampled(oracle, s, pr.P, pr.D, pb, label="2048^2 order 8")


def test_fp32_flux_order8_error_report(oracle):
    """The FP32 gas-kinetic variant with the order-8 flux (FP64 assembly and
    update): one stage against the FP64 oracle, reported, and held to the
    error level of the FP32 variant with the order-6 flux."""
    s, P, D = CASES["shear_ns_36"]()
    par = oracle_par(oracle, s)
    dt = 0.2 * (s["lx"] / s["nx"]) / 3.0
    oP, oD, _, _ = oracle.stage2d(par, 1, dt, P, D)
    fl = _floors(s, P, D)
    err = {}
    for order in (6, 8):
        so = dict(s, flux_order=order, fp32_flux=True)
        g1, _ = _problem(so, P, D).debug_stage(1, dt)
        ref = (oP, oD) if order == 8 else oracle.stage2d(oracle_par(oracle, dict(s, flux_order=6)), 1, dt, P, D)[:2]
        err[order] = max(relerr(g1[g][:4], ref[g][:4], fl[:4])[0] for g in (0, 1))
    print(f"FP32-flux stage-1 max-relative error on values: order 6 {err[6]:.3e}, order 8 {err[8]:.3e}")
    assert err[8] < 1e-5 and err[8] < 10 * err[6]


# ----------------------------------------------------------------------- 1D
CASES1D = {
    "rough_77": lambda: (settings(dim=1, nx=77, lx=1.0, flux_order=8), T1._rough1d(77, 5)),
    "advection_100_dual": lambda: (settings(dim=1, nx=100, lx=2.0, dual_1d=1, flux_order=8),
                                   WL.advection1d(100, seed=1).S),
    "tube_400_zero_gradient": lambda: (settings(dim=1, nx=400, lx=1.0, bc="zero_gradient", flux_order=8),
                                       WL.seeded_shock_tube(400, 2).S),
    "mirror_60_reflecting": lambda: (settings(dim=1, nx=60, lx=1.0, bc="reflecting", flux_order=8),
                                     TB._mirror_line(60)),
}


@pytest.mark.parametrize("name", list(CASES1D))
def test_stages_1d_order8(oracle, name):
    s, S = CASES1D[name]()
    print(f"order-8 1D stages: {name}", flush=True)
    par = oracle_par(oracle, s)
    dt = 0.2 * (s["lx"] / s["nx"]) / 3.0
    o1, a1 = oracle.stage1d(par, 1, dt, S)
    o2 = oracle.stage1d(par, 2, dt, o1, a1)
    pb = T1._problem(s, S)
    fl = T1._floors(S, L=s["lx"])
    g1, ga = pb.debug_stage(1, dt)
    for g, o in ((g1.reshape(S.shape), o1), (ga.reshape(S.shape), a1)):
        err, where = relerr(g, o, fl, ndim_plane=1)
        assert err <= TOL, (where, err)
    err, where = relerr(pb.debug_stage(2, dt).reshape(S.shape), o2, fl, ndim_plane=1)
    assert err <= TOL, (where, err)


def test_order_of_accuracy_1d():
    """Smooth advection to t = 2 with dt ~ h^2 (the setup of the accuracy
    test of Sec. 5.1) through the GPU path: with flux_order 8 the L1 error
    falls by more than 2^7 per mesh halving and stays below the order-6
    error; the order-6 flux converges at about 6."""
    errs = {6: [], 8: []}
    for order in (6, 8):
        for N in (8, 16, 32):
            h = 2.0 / N
            S = WL.advection1d(N, noise=0, dual=False).S
            s = settings(dim=1, nx=N, lx=2.0, variant="6-2", flux_order=order)
            pb = T1._problem(s, S)
            dt = 0.1 * h * (h / 0.25) / (1 + np.sqrt(1.4 / 0.8))
            nst = int(np.ceil(2.0 / dt))
            t, n = pb.step(nsteps=nst, dt=2.0 / nst)
            assert n == nst and abs(t - 2.0) < 1e-12
            rho = pb.get_state_stacked(0).reshape(6, N)[0]
            errs[order].append(float(np.abs(rho - WL.advection1d_exact(N, 2.0)[0]).mean()))
    rates = {o: [np.log2(a / b) for a, b in zip(e, e[1:])] for o, e in errs.items()}
    print("L1 errors", errs, "rates", rates)
    assert all(r > 7.0 for r in rates[8]) and all(5.5 < r < 7.0 for r in rates[6])
    assert errs[8][2] < 0.2 * errs[6][2]
