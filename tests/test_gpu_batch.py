"""Batched 2D solves over many uneven grids, in every launch mode (one launch
per phase, also captured as HIP graphs; one cooperative persistent launch per
stage), with periodic and bounded members and each scheme option
(characteristic reconstruction, order-8 flux), against the single-problem HIP
path and the oracle (GPU)."""
import numpy as np
import pytest

import workloads as WL
from tests.helpers import TOL, floors_state, gpu_params, oracle_par, ref_scales, relerr, settings, ulp_sensitivity

pytestmark = pytest.mark.gpu


def _members(sizes, seed=0):
    probs = []
    for b, n in enumerate(sizes):
        probs.append(WL.vortex(n, seed=seed + b) if b % 2 == 0 else WL.riemann2d(n, seed=seed + b))
    return probs


def _settings(pr):
    return settings(dim=2, nx=pr.nx, ny=pr.ny, lx=pr.lx)


MODES = ["phased", "persistent", "graph"]


def _batch(probs, mode, setts=None):
    from paper_2606_17772_amd import Batch
    B = Batch([gpu_params(s) for s in (setts or [_settings(p) for p in probs])])
    B.set_mode(mode)
    return B


def _bounded_members():
    """Members with bounded sides: zero-gradient four-quadrant Riemann data,
    a no-slip / reflecting Navier-Stokes flow, mixed sides, and a periodic
    vortex beside them."""
    out = []
    pr = WL.riemann2d_bounded(21, seed=3)
    out.append((settings(dim=2, nx=21, ny=21, lx=1.0, bc="zero_gradient"), pr.P, pr.D))
    P, D = WL.sample_bounded(WL.mirror_flow(1.0, 0.5, 1, 1), 30, 15, 1.0 / 30, 1, 1)
    out.append((settings(dim=2, nx=30, ny=15, lx=1.0, mu=0.0, sides=["no_slip", "no_slip", "reflecting",
                                                                     "reflecting"]), P, D))
    P, D = WL.sample_bounded(WL.mirror_flow(1.0, 20 / 48, 1, 1), 48, 20, 1.0 / 48, 1, 1)
    out.append((settings(dim=2, nx=48, ny=20, lx=1.0, sides=["reflecting", "zero_gradient", "zero_gradient",
                                                             "reflecting"]), P, D))
    v = WL.vortex(26, seed=5)
    out.append((_settings(v), v.P, v.D))
    pr = WL.riemann2d_bounded(67, seed=4)
    out.append((settings(dim=2, nx=67, ny=67, lx=1.0, bc="zero_gradient"), pr.P, pr.D))
    return out


@pytest.mark.parametrize("mode", MODES)
def test_batch_matches_single_problem_path_bitwise(mode):
    """Every member of a batch of uneven grids (including ragged tile edges)
    is bitwise identical to the same problem run alone (same device
    arithmetic, per-member CFL time step)."""
    from paper_2606_17772_amd import Problem
    sizes = [16, 37, 64, 23, 90, 8]
    probs = _members(sizes)
    B = _batch(probs, mode)
    for m, p in enumerate(probs):
        B.set_state_stacked(m, 0, p.P)
        B.set_state_stacked(m, 1, p.D)
    t, dt, n = B.step(nsteps=3, cfl=0.5)
    assert n == 3
    for m, p in enumerate(probs):
        pb = Problem(gpu_params(_settings(p)))
        pb.set_state_stacked(0, p.P)
        pb.set_state_stacked(1, p.D)
        ts, ns = pb.step(nsteps=3, cfl=0.5)
        assert ns == 3 and t[m] == ts, (m, t[m], ts)
        for g in (0, 1):
            assert np.array_equal(B.get_state_stacked(m, g), pb.get_state_stacked(g)), (m, g)


@pytest.mark.parametrize("mode", MODES)
def test_batch_against_oracle(mode):
    from oracle import oracle as O
    sizes = [20, 33, 12]
    probs = _members(sizes, seed=7)
    B = _batch(probs, mode)
    for m, p in enumerate(probs):
        B.set_state_stacked(m, 0, p.P)
        B.set_state_stacked(m, 1, p.D)
    t, dt, n = B.step(nsteps=2, cfl=0.5)
    for m, p in enumerate(probs):
        s = _settings(p)
        par = oracle_par(O, s)
        oP, oD, ot, ok = O.step2d(par, p.P, p.D, 2, cfl=0.5)
        assert abs(t[m] - ot) <= 1e-13 * ot
        fl = floors_state(ref_scales([p.P, p.D], 1.4, p.lx))
        sens = ulp_sensitivity(lambda P, D: O.step2d(par, P, D, 2, cfl=0.5)[:2], p.P, p.D, fl)
        for g, o in ((B.get_state_stacked(m, 0), oP), (B.get_state_stacked(m, 1), oD)):
            err, where = relerr(g, o, fl)
            assert err <= max(TOL, 4 * sens), (m, where, err, sens)


@pytest.mark.parametrize("mode", MODES)
def test_batch_nonphysical_member_stops_and_rolls_back(mode):
    from paper_2606_17772_amd import FdcgksError
    probs = _members([16, 20])
    P = probs[1].P.copy()
    P[3, 5, 5] = -1.0  # negative energy -> p < 0
    B = _batch(probs, mode)
    B.set_state_stacked(0, 0, probs[0].P)
    B.set_state_stacked(0, 1, probs[0].D)
    B.set_state_stacked(1, 0, P)
    B.set_state_stacked(1, 1, probs[1].D)
    with pytest.raises(FdcgksError) as ei:
        B.step(nsteps=2, cfl=0.5)
    assert ei.value.status == -4 and "member 1" in str(ei.value)
    assert np.array_equal(B.get_state_stacked(0, 0), probs[0].P)
    assert np.array_equal(B.get_state_stacked(1, 0), P)


@pytest.mark.parametrize("mode", MODES + ["single"])
def test_failure_in_stage_two_rolls_back(mode):
    """Four-quadrant data (seed 1, 16^2) at CFL 1.2: stage 1 stays physical
    (oracle: min p 0.35) and stage 2 does not (oracle: min p -0.27).  The
    failing step is not counted, the state is the step's input, and a later
    step at a stable CFL proceeds from it."""
    from paper_2606_17772_amd import FdcgksError, Problem
    pr = WL.riemann2d(16, seed=1)
    if mode == "single":
        pb = Problem(gpu_params(_settings(pr)))
        pb.set_state_stacked(0, pr.P)
        pb.set_state_stacked(1, pr.D)
        with pytest.raises(FdcgksError) as ei:
            pb.step(nsteps=3, cfl=1.2)
        got = [pb.get_state_stacked(g) for g in (0, 1)]
        t, n = pb.step(nsteps=1, cfl=0.4)
    else:
        B = _batch([pr], mode)
        B.set_state_stacked(0, 0, pr.P)
        B.set_state_stacked(0, 1, pr.D)
        with pytest.raises(FdcgksError) as ei:
            B.step(nsteps=3, cfl=1.2)
        got = [B.get_state_stacked(0, g) for g in (0, 1)]
        _, _, n = B.step(nsteps=1, cfl=0.4)
    assert ei.value.status == -4 and "step 1 stage 2" in str(ei.value), str(ei.value)
    assert np.array_equal(got[0], pr.P) and np.array_equal(got[1], pr.D)
    assert n == 1


@pytest.mark.parametrize("mode", MODES)
def test_bounded_members_match_single_problems_bitwise(mode):
    """Members with zero-gradient, reflecting and no-slip sides (their dual
    grids carry the boundary nodes) advance bit for bit like the same
    problems alone; 18 steps, so that the graph mode replays a captured
    graph and launches the remainder."""
    from paper_2606_17772_amd import Problem
    mem = _bounded_members()
    B = _batch(None, mode, [m[0] for m in mem])
    for k, (s, P, D) in enumerate(mem):
        B.set_state_stacked(k, 0, P)
        B.set_state_stacked(k, 1, D)
    t, dt, n = B.step(nsteps=18, cfl=0.4)
    assert n == 18
    for k, (s, P, D) in enumerate(mem):
        pb = Problem(gpu_params(s))
        pb.set_state_stacked(0, P)
        pb.set_state_stacked(1, D)
        ts, ns = pb.step(nsteps=18, cfl=0.4)
        assert ns == 18 and t[k] == ts, (k, t[k], ts)
        for g in (0, 1):
            assert np.array_equal(B.get_state_stacked(k, g), pb.get_state_stacked(g)), (k, g)


SCHEMES = {"char": dict(recon_vars="characteristic"), "order8": dict(flux_order=8),
           "char_order8": dict(recon_vars="characteristic", flux_order=8)}


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("scheme", list(SCHEMES))
def test_scheme_options_match_single_problems_bitwise(mode, scheme):
    """Characteristic reconstruction and the order-8 compact flux in a batch:
    periodic and bounded members of uneven sizes advance bit for bit like the
    same problems alone (18 steps: the graph mode replays a captured graph
    and launches the remainder).  The single-problem path of each option is
    held to the oracle by its own tests."""
    from paper_2606_17772_amd import Problem
    kw = SCHEMES[scheme]
    mem = [(_settings(p), p.P, p.D) for p in _members([16, 37, 23], seed=21)] + _bounded_members()
    mem = [(dict(s, **kw), P, D) for s, P, D in mem]
    B = _batch(None, mode, [m[0] for m in mem])
    for k, (s, P, D) in enumerate(mem):
        B.set_state_stacked(k, 0, P)
        B.set_state_stacked(k, 1, D)
    t, dt, n = B.step(nsteps=18, cfl=0.4)
    assert n == 18
    for k, (s, P, D) in enumerate(mem):
        pb = Problem(gpu_params(s))
        pb.set_state_stacked(0, P)
        pb.set_state_stacked(1, D)
        ts, ns = pb.step(nsteps=18, cfl=0.4)
        assert ns == 18 and t[k] == ts, (k, t[k], ts)
        for g in (0, 1):
            assert np.array_equal(B.get_state_stacked(k, g), pb.get_state_stacked(g)), (scheme, k, g)


def test_scheme_options_must_agree_across_members():
    """One batch runs one scheme: members that differ in reconstruction
    variables or flux order are rejected at creation."""
    from paper_2606_17772_amd import Batch, FdcgksError
    a = _settings(WL.vortex(16, seed=1))
    for kw in SCHEMES.values():
        with pytest.raises(FdcgksError, match="scheme constants differ"):
            Batch([gpu_params(a), gpu_params(dict(a, **kw))])


def test_bounded_members_against_oracle():
    """Zero-gradient Riemann and walled members against the oracle, two CFL
    steps (bar: max(1e-12, 4 x the oracle's one-ulp sensitivity))."""
    from oracle import oracle as O
    mem = _bounded_members()
    B = _batch(None, "graph", [m[0] for m in mem])
    for k, (s, P, D) in enumerate(mem):
        B.set_state_stacked(k, 0, P)
        B.set_state_stacked(k, 1, D)
    t, dt, n = B.step(nsteps=2, cfl=0.4)
    for k, (s, P, D) in enumerate(mem):
        par = oracle_par(O, s)
        oP, oD, ot, ok = O.step2d(par, P, D, 2, cfl=0.4)
        assert ok == 2 and abs(t[k] - ot) <= 1e-13 * ot
        fl = floors_state(ref_scales([P, D], 1.4, s["lx"]))
        sens = ulp_sensitivity(lambda A, C: O.step2d(par, A, C, 2, cfl=0.4)[:2], P, D, fl)
        for g, o in ((B.get_state_stacked(k, 0), oP), (B.get_state_stacked(k, 1), oD)):
            err, where = relerr(g, o, fl)
            print(f"member {k} grid: gpu-oracle {err:.2e}, oracle 1-ulp sensitivity {sens:.2e}")
            assert err <= max(TOL, 4 * sens), (k, where, err, sens)


def test_graph_mode_replays_equal_separate_launches():
    """40 steps (two captured 16-step graphs and 8 separate steps), then 16
    more from the other parity, against the same steps launched separately;
    every replay is checked after the program's own synchronising reads."""
    sizes = [16, 37, 64, 23]
    probs = _members(sizes, seed=11)
    A = _batch(probs, "graph")
    C = _batch(probs, "phased")
    for m, p in enumerate(probs):
        for B in (A, C):
            B.set_state_stacked(m, 0, p.P)
            B.set_state_stacked(m, 1, p.D)
    for steps in (40, 16, 33):
        ta, _, na = A.step(nsteps=steps, cfl=0.4)
        tc, _, nc = C.step(nsteps=steps, cfl=0.4)
        assert na == nc == steps and np.array_equal(ta, tc)
        for m in range(len(probs)):
            for g in (0, 1):
                assert np.array_equal(A.get_state_stacked(m, g), C.get_state_stacked(m, g)), (steps, m, g)
