"""Batched 2D solves over many uneven grids, in both launch modes (one launch
per phase; one cooperative persistent launch per stage), against the
single-problem HIP path and the oracle (GPU)."""
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


MODES = ["phased", "persistent"]


def _batch(probs, mode):
    from paper_2606_17772_amd import Batch
    B = Batch([gpu_params(_settings(p)) for p in probs])
    B.set_mode(mode)
    return B


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
