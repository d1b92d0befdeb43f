"""Parity of the HIP path's characteristic-variable reconstruction (Sec. 3:
Q a characteristic component; eigenvectors at the mean interface state, chi
from the u -/+ c fields) against the oracle in the same mode (GPU).

Same cases and bars as the conservative-variable parity tests: interface and
node intermediates and both stages at the floored 1e-12 bar, several CFL
steps at max(1e-12, 4 x the oracle's one-ulp sensitivity), 1D stages at
1e-12, sampled nodes of one step at the full 2048^2 size in the benchmark's
launch shapes.  Batches and the step adjoint in this mode: test_gpu_batch.py,
test_gpu_adjoint.py."""
import numpy as np
import pytest

import workloads as WL
from tests.helpers import (TOL, check_edge_intermediates, floors_edge, floors_node, floors_state,
                           check_full_size_sampled, gpu_params, oracle_par, ref_scales, relerr, settings,
                           ulp_sensitivity)
from tests.test_gpu_parity1d import CASES as CASES1D
from tests.test_gpu_parity1d import _floors as _floors1d
from tests.test_gpu_parity2d import _bench_tiles
from tests.test_gpu_parity2d import _case as _case2d

pytestmark = pytest.mark.gpu

CHAR = dict(recon_vars="characteristic")
NAMES2D = ["smooth_70x37", "rough_67x9", "vortex_40", "shear_ns_36", "riemann_33x20"]


def _case(name):
    s, pr = _case2d(name)
    return dict(s, **CHAR), pr


def _problem(s, P, D):
    from paper_2606_17772_amd import Problem
    pb = Problem(gpu_params(s))
    pb.set_state_stacked(0, P)
    pb.set_state_stacked(1, D)
    return pb


@pytest.mark.parametrize("name", NAMES2D)
def test_intermediates_char(oracle, name):
    """Every plane at the 1e-12 bar except chi, held to the oracle's one-ulp
    sensitivity (the two sides also round the eigenvector products
    differently: Gauss-Jordan against the closed form)."""
    s, pr = _case(name)
    dt = 0.2 * pr.h / 3.0
    par = oracle_par(oracle, s)
    X, Y, NP, ND = oracle.intermediates2d(par, dt, pr.P, pr.D)
    gx, gy, gp, gd = _problem(s, pr.P, pr.D).debug_intermediates(dt)
    sc = ref_scales([pr.P, pr.D], s["gamma"], s["lx"])
    check_edge_intermediates(oracle, par, dt, pr.P, pr.D, (gx, gy), (X, Y), floors_edge(sc), name)
    for lab, g, o in (("nodeP", gp, NP), ("nodeD", gd, ND)):
        err, where = relerr(g, o, floors_node(sc))
        assert err <= TOL, (lab, where, err)


@pytest.mark.parametrize("name", NAMES2D)
def test_stages_char(oracle, name):
    s, pr = _case(name)
    dt = 0.2 * pr.h / 3.0
    par = oracle_par(oracle, s)
    oP, oD, aP, aD = oracle.stage2d(par, 1, dt, pr.P, pr.D)
    o2P, o2D = oracle.stage2d(par, 2, dt, oP, oD, aP, aD)
    pb = _problem(s, pr.P, pr.D)
    fl = floors_state(ref_scales([pr.P, pr.D], s["gamma"], s["lx"]))
    g1, ga = pb.debug_stage(1, dt)
    for g, o in ((g1[0], oP), (g1[1], oD), (ga[0], aP), (ga[1], aD)):
        err, where = relerr(g, o, fl)
        assert err <= TOL, (where, err)
    g2 = pb.debug_stage(2, dt)
    for g, o in ((g2[0], o2P), (g2[1], o2D)):
        err, where = relerr(g, o, fl)
        assert err <= TOL, (where, err)


def test_modes_differ_where_the_path_function_acts(oracle):
    """The GPU's characteristic result is not the conservative one on data
    with a discontinuity (the mode switch reaches the kernels)."""
    s, pr = _case("riemann_33x20")
    dt = 0.2 * pr.h / 3.0
    a = _problem(s, pr.P, pr.D).debug_stage(1, dt)[0]
    b = _problem(dict(s, recon_vars="conservative"), pr.P, pr.D).debug_stage(1, dt)[0]
    assert np.abs(a - b).max() > 1e-6 * np.abs(b).max()


@pytest.mark.parametrize("name,nsteps", [("vortex_40", 3), ("riemann_33x20", 2), ("shear_ns_36", 3)])
def test_steps_cfl_char(oracle, name, nsteps):
    s, pr = _case(name)
    par = oracle_par(oracle, s)
    pb = _problem(s, pr.P, pr.D)
    oP, oD, ot, ok = oracle.step2d(par, pr.P, pr.D, nsteps, dt=0.0, cfl=0.5)
    t, n = pb.step(nsteps=nsteps, cfl=0.5)
    assert n == nsteps == ok
    assert abs(t - ot) <= 1e-13 * ot
    fl = floors_state(ref_scales([pr.P, pr.D], s["gamma"], s["lx"]))
    sens = ulp_sensitivity(lambda P, D: oracle.step2d(par, P, D, nsteps, dt=0.0, cfl=0.5)[:2], pr.P, pr.D, fl)
    for g, o in ((pb.get_state_stacked(0), oP), (pb.get_state_stacked(1), oD)):
        err, where = relerr(g, o, fl)
        print(f"{name} {nsteps} characteristic steps: gpu-oracle {err:.2e}, oracle 1-ulp sensitivity {sens:.2e}")
        assert err <= max(TOL, 4 * sens), (where, err, sens)


def test_captured_and_fused_steps_char(oracle):
    """Steps replayed from captured graphs, and steps with the node sweep
    fused into the update kernel, match eager unfused steps bit for bit."""
    s, pr = _case("vortex_40")
    a = _problem(s, pr.P, pr.D)
    a.use_graph = False
    a.step(nsteps=5, cfl=0.5)
    b = _problem(s, pr.P, pr.D)
    b.graph_steps = 4
    b.step(nsteps=5, cfl=0.5)
    c = _problem(s, pr.P, pr.D)
    c.use_graph = False
    c.fuse_stage = False  # the stage fusion takes precedence over the node fusion
    c.fuse_nodes = True
    c.step(nsteps=5, cfl=0.5)
    for g in (0, 1):
        assert np.array_equal(a.get_state_stacked(g), b.get_state_stacked(g))
        assert np.array_equal(a.get_state_stacked(g), c.get_state_stacked(g))


def test_fp32_flux_char_error_report(oracle):
    s, pr = _case("vortex_40")
    par = oracle_par(oracle, s)
    dt = 0.2 * pr.h / 3.0
    oP, _, _, _ = oracle.stage2d(par, 1, dt, pr.P, pr.D)
    g1, _ = _problem(dict(s, fp32_flux=True), pr.P, pr.D).debug_stage(1, dt)
    fl = floors_state(ref_scales([pr.P, pr.D], s["gamma"], s["lx"]))
    errW = relerr(g1[0][:4], oP[:4], fl[:4])[0]
    errG = relerr(g1[0][4:], oP[4:], fl[4:])[0]
    print(f"FP32-flux characteristic stage-1 max-relative error: values {errW:.3e}, gradients {errG:.3e}")
    assert errW < 1e-5 and errG < 1e-3


def test_full_size_sampled_char(oracle):
    """One step of the 2048^2 shear layer in characteristic mode, in the
    benchmark's launch shapes, on sampled nodes (bars: check_full_size_sampled)."""
    n = 2048
    pr = WL.shear_layer(n, seed=0)
    s = settings(dim=2, nx=n, ny=n, lx=1.0, mu=1e-4, prandtl=0.72, **CHAR)
    pb = _problem(s, pr.P, pr.D)
    _bench_tiles(pb)
    check_full_size_sampled(oracle, s, pr.P, pr.D, pb, ns=32, seed=1, label="2048^2 characteristic")


@pytest.mark.parametrize("name", list(CASES1D))
def test_stages_1d_char(oracle, name):
    s, S = CASES1D[name]()
    s = dict(s, **CHAR)
    par = oracle_par(oracle, s)
    dt = 0.2 * s["lx"] / s["nx"] / 3.0
    o1, a1 = oracle.stage1d(par, 1, dt, S)
    o2 = oracle.stage1d(par, 2, dt, o1, a1)
    from paper_2606_17772_amd import Problem
    pb = Problem(gpu_params(s))
    for g in range(S.shape[0]):
        pb.set_state_stacked(g, S[g])
    fl = _floors1d(S, L=s["lx"])
    g1, ga = pb.debug_stage(1, dt)
    for g, o in ((g1.reshape(S.shape), o1), (ga.reshape(S.shape), a1)):
        err, where = relerr(g, o, fl, ndim_plane=1)
        assert err <= TOL, (where, err)
    err, where = relerr(pb.debug_stage(2, dt).reshape(S.shape), o2, fl, ndim_plane=1)
    assert err <= TOL, (where, err)


@pytest.mark.parametrize("name,t_end", [("sod_100_62", 0.2), ("advection_100_dual", 2.0)])
def test_long_run_1d_char(oracle, name, t_end):
    """Whole 1D runs in one launch (chaotic in round-off: shocks, grid-scale
    noise): same step count and end time as the oracle, and the L1 distance
    of the values within 4x the oracle's own one-ulp spread in that norm."""
    s, S = CASES1D[name]()
    s = dict(s, **CHAR)
    par = oracle_par(oracle, s)
    run = lambda X: oracle.step1d(par, X, 100000, cfl=0.5, t_end=t_end)[0]  # noqa: E731
    oS, ot, ok = oracle.step1d(par, S, 100000, cfl=0.5, t_end=t_end)
    from paper_2606_17772_amd import Problem
    pb = Problem(gpu_params(s))
    for g in range(S.shape[0]):
        pb.set_state_stacked(g, S[g])
    t, n = pb.step(nsteps=100000, cfl=0.5, t_end=t_end)
    assert n == ok and abs(t - t_end) < 1e-14
    g = np.stack([pb.get_state_stacked(k).reshape(6, -1) for k in range(S.shape[0])])
    l1 = lambda A, B: float(np.abs(A[:, :3] - B[:, :3]).mean() / np.abs(B[:, :3]).mean())  # noqa: E731
    rng = np.random.default_rng(0)
    spread = max(l1(run(S * (1 + np.finfo(float).eps * rng.choice([-1.0, 1.0], size=S.shape))), oS)
                 for _ in range(4))
    err = l1(g, oS)
    print(f"{name} characteristic: {n} steps, values L1 gpu-oracle {err:.2e}, oracle one-ulp spread {spread:.2e}")
    assert err <= max(TOL, 4 * spread)
