"""2D parity of the HIP path against the oracle (GPU).

Same seeded inputs on both sides; comparisons element by element on whole
grids at sizes the oracle finishes in seconds (several 64-wide tiles and a
ragged tail in x and y), and on sampled nodes at the full 2048^2 size.
Bar: per-plane max |gpu - oracle| / max(max |oracle|, floor) <= 1e-12 (FP64), the floor being
the dimensional reference scale of the field (tests/helpers.py).
"""
import pytest

import workloads as WL
from tests.helpers import (TOL, check_edge_intermediates, check_full_size_sampled, floors_edge, floors_node,
                           floors_state, gpu_params, oracle_par, ref_scales, relerr, settings, ulp_sensitivity)

pytestmark = pytest.mark.gpu


def _problem(s, P, D):
    from paper_2606_17772_amd import Problem
    pb = Problem(gpu_params(s))
    pb.set_state_stacked(0, P)
    pb.set_state_stacked(1, D)
    return pb


CASES = {
    "smooth_70x37": lambda: (settings(dim=2, nx=70, ny=37, lx=1.0), WL.random_smooth2d(70, 37, seed=3)),
    "rough_67x9": lambda: (settings(dim=2, nx=67, ny=9, lx=1.0), WL.random_rough2d(67, 9, seed=4)),
    "vortex_40": lambda: (settings(dim=2, nx=40, ny=40, lx=10.0), WL.vortex(40, seed=1)),
    "shear_ns_36": lambda: (settings(dim=2, nx=36, ny=36, lx=1.0, mu=1e-3, prandtl=0.72),
                            WL.shear_layer(36, seed=2, k=20.0)),
    "riemann_33x20": lambda: (settings(dim=2, nx=33, ny=20, lx=1.0), WL.riemann2d(33, seed=5)),
    "riemann_33x20_62": lambda: (settings(dim=2, nx=33, ny=20, lx=1.0, variant="6-2"), WL.riemann2d(33, seed=6)),
    "rough_67x9_linear": lambda: (settings(dim=2, nx=67, ny=9, lx=1.0, variant="linear"),
                                  WL.random_rough2d(67, 9, seed=7)),
}


def _case(name):
    s, pr = CASES[name]()
    if pr.ny != s["ny"]:
        pr = WL.Problem2D(pr.name, s["nx"], s["ny"], 0, s["lx"], 0, s["lx"] * s["ny"] / s["nx"],
                          pr.P[:, :s["ny"]], pr.D[:, :s["ny"]])
    return s, pr


ALL = list(CASES)


@pytest.mark.parametrize("name", ALL)
def test_intermediates(oracle, name):
    s, pr = _case(name)
    dt = 0.2 * pr.h / 3.0
    par = oracle_par(oracle, s)
    X, Y, NP, ND = oracle.intermediates2d(par, dt, pr.P, pr.D)
    pb = _problem(s, pr.P, pr.D)
    gx, gy, gp, gd = pb.debug_intermediates(dt)
    sc = ref_scales([pr.P, pr.D], s["gamma"], s["lx"])
    check_edge_intermediates(oracle, par, dt, pr.P, pr.D, (gx, gy), (X, Y), floors_edge(sc), name)
    for lab, g, o, fl in (("nodeP", gp, NP, floors_node(sc)), ("nodeD", gd, ND, floors_node(sc))):
        err, where = relerr(g, o, fl)
        assert err <= TOL, (lab, where, err)


@pytest.mark.parametrize("name", ALL)
def test_stages(oracle, name):
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


@pytest.mark.parametrize("name,nsteps", [("vortex_40", 3), ("shear_ns_36", 3), ("riemann_33x20", 2),
                                         ("smooth_70x37", 3), ("riemann_33x20_62", 2)])
def test_steps_cfl(oracle, name, nsteps):
    """Several CFL steps.  Over several steps the nonlinear weights amplify
    round-off (near discontinuities by ~20x per step), so the bar is
    max(1e-12, 4 x the oracle's own change under a one-ulp input
    perturbation), measured here on the same case."""
    s, pr = _case(name)
    par = oracle_par(oracle, s)
    dt0 = oracle.dt2d(par, pr.P, pr.D, 0.5)
    pb = _problem(s, pr.P, pr.D)
    assert abs(pb.compute_dt(0.5) - dt0) <= 1e-14 * dt0
    oP, oD, ot, ok = oracle.step2d(par, pr.P, pr.D, nsteps, dt=0.0, cfl=0.5)
    t, n = pb.step(nsteps=nsteps, cfl=0.5)
    assert n == nsteps == ok
    assert abs(t - ot) <= 1e-13 * ot
    fl = floors_state(ref_scales([pr.P, pr.D], s["gamma"], s["lx"]))
    sens = ulp_sensitivity(lambda P, D: oracle.step2d(par, P, D, nsteps, dt=0.0, cfl=0.5)[:2], pr.P, pr.D, fl)
    bar = max(TOL, 4 * sens)
    for g, o in ((pb.get_state_stacked(0), oP), (pb.get_state_stacked(1), oD)):
        err, where = relerr(g, o, fl)
        print(f"{name} {nsteps} steps: gpu-oracle {err:.2e}, oracle 1-ulp sensitivity {sens:.2e}")
        assert err <= bar, (where, err, sens)


def test_t_end_clip(oracle):
    s, pr = _case("vortex_40")
    par = oracle_par(oracle, s)
    dt = 0.01
    oP, oD, ot, ok = oracle.step2d(par, pr.P, pr.D, 10, dt=dt, t_end=0.025)
    pb = _problem(s, pr.P, pr.D)
    t, n = pb.step(nsteps=10, dt=dt, t_end=0.025)
    assert n == ok == 3 and abs(t - 0.025) < 1e-15
    fl = floors_state(ref_scales([pr.P, pr.D], s["gamma"], s["lx"]))
    assert relerr(pb.get_state_stacked(0), oP, fl)[0] <= TOL
    assert relerr(pb.get_state_stacked(1), oD, fl)[0] <= TOL


def _bench_tiles(pb):
    """The launch shapes the benchmark times."""
    import bench
    for item in bench.DEFAULT_TILES.split(","):
        name, xy = item.split("=")
        pb.set_tile(name, *(int(v) for v in xy.split("x")))


def test_vortex_512_steps(oracle):
    """2D Euler isentropic vortex at its benchmark size, 512^2 + dual: three
    CFL-0.5 steps compared on every node (values and averaged gradients)
    against the oracle, bar max(1e-12, 4 x the oracle's one-ulp
    sensitivity over the same steps)."""
    n = 512
    pr = WL.vortex(n, seed=0)
    s = settings(dim=2, nx=n, ny=n, lx=10.0)
    par = oracle_par(oracle, s)
    pb = _problem(s, pr.P, pr.D)
    _bench_tiles(pb)
    t, k = pb.step(nsteps=3, cfl=0.5)
    run = lambda P, D: oracle.step2d(par, P, D, 3, cfl=0.5)[:2]  # noqa: E731
    oP, oD, ot, ok = oracle.step2d(par, pr.P, pr.D, 3, cfl=0.5)
    assert k == ok == 3 and abs(t - ot) <= 1e-14 * ot
    fl = floors_state(ref_scales([pr.P, pr.D], s["gamma"], s["lx"]))
    sens = ulp_sensitivity(run, pr.P, pr.D, fl, trials=1)
    err = max(relerr(pb.get_state_stacked(0), oP, fl)[0], relerr(pb.get_state_stacked(1), oD, fl)[0])
    print(f"vortex 512^2, 3 steps: gpu-oracle {err:.2e}, oracle 1-ulp sensitivity {sens:.2e}")
    assert err <= max(TOL, 4 * sens), (err, sens)


def test_full_size_sampled(oracle):
    """One full step on the 2048^2 shear-layer workload in the launch
    configuration the benchmark times, checked on sampled nodes (bars:
    check_full_size_sampled)."""
    n = 2048
    pr = WL.shear_layer(n, seed=0)
    s = settings(dim=2, nx=n, ny=n, lx=1.0, mu=1e-4, prandtl=0.72)
    pb = _problem(s, pr.P, pr.D)
    _bench_tiles(pb)
    check_full_size_sampled(oracle, s, pr.P, pr.D, pb, label="2048^2 shear layer")
