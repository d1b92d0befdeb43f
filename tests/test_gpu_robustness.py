"""Diagnostics, determinism and failure handling of the 2D path (GPU).

Failures are forced from the host (a NaN or a negative pressure in the
state, a time step far beyond the stable one): every kernel still runs to
completion; the step reports ENONPHYS and the state stays at the last good
step."""
import numpy as np
import pytest

import workloads as WL
from tests.helpers import gpu_params, settings

pytestmark = pytest.mark.gpu

ENONPHYS = -4


def _problem(s, P, D):
    from paper_2606_17772_amd import Problem
    pb = Problem(gpu_params(s))
    pb.set_state_stacked(0, P)
    pb.set_state_stacked(1, D)
    return pb


def _pressure(A, gamma=1.4):
    W = A[:4]
    return (gamma - 1) * (W[3] - 0.5 * (W[1] ** 2 + W[2] ** 2) / W[0])


@pytest.mark.parametrize("bounded", [False, True])
def test_diagnostics_match_the_state(bounded):
    if bounded:
        n = 40
        P, D = WL.sample_bounded(WL.mirror_flow(1.0, 1.0, 1, 1), n, n, 1.0 / n, 1, 1)
        s = settings(dim=2, nx=n, ny=n, lx=1.0, bc="reflecting")
    else:
        pr = WL.vortex(40, seed=3)
        P, D = pr.P, pr.D
        s = settings(dim=2, nx=40, ny=40, lx=10.0)
    pb = _problem(s, P, D)
    pb.step(nsteps=2, cfl=0.5)
    d = pb.diagnostics()
    G = [pb.get_state_stacked(0), pb.get_state_stacked(1)]
    for g in range(2):
        ref = G[g][:4].reshape(4, -1).sum(axis=1)
        assert np.allclose(d["sums"][g], ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    assert d["rho_min"] == min(G[0][0].min(), G[1][0].min())
    pmin = min(_pressure(G[0]).min(), _pressure(G[1]).min())
    assert abs(d["p_min"] - pmin) <= 1e-14 * abs(pmin)
    assert pb.diagnostics()["sums"].tobytes() == d["sums"].tobytes()


def test_diagnostics_1d():
    from paper_2606_17772_amd import Problem
    S = WL.advection1d(100, seed=0).S
    pb = Problem(gpu_params(settings(dim=1, nx=100, lx=2.0, dual_1d=1)))
    for g in range(2):
        pb.set_state_stacked(g, S[g])
    d = pb.diagnostics()
    for g in range(2):
        assert np.allclose(d["sums"][g], S[g, :3].sum(axis=1), rtol=1e-13)
    assert d["rho_min"] == S[:, 0].min()


def test_repeated_runs_are_bitwise_equal():
    pr = WL.riemann2d(48, seed=2)
    s = settings(dim=2, nx=48, ny=48, lx=1.0)
    pb = _problem(s, pr.P, pr.D)
    pb.step(nsteps=5, cfl=0.5)
    a = [pb.get_state_stacked(g) for g in range(2)]
    pb.set_state_stacked(0, pr.P)
    pb.set_state_stacked(1, pr.D)
    pb.step(nsteps=5, cfl=0.5)
    for g in range(2):
        assert np.array_equal(a[g], pb.get_state_stacked(g))


@pytest.mark.parametrize("how", ["nan", "negative_pressure", "huge_dt"])
def test_non_physical_step_rolls_back(how):
    from paper_2606_17772_amd import FdcgksError
    pr = WL.vortex(32, seed=1)
    s = settings(dim=2, nx=32, ny=32, lx=10.0)
    P, D = pr.P.copy(), pr.D.copy()
    if how == "nan":
        D[1, 7, 11] = np.nan
    elif how == "negative_pressure":
        P[3, 20, 5] = 0.1 * P[3, 20, 5] - 10.0
    pb = _problem(s, P, D)
    good = 0
    if how == "huge_dt":
        pb.step(nsteps=2, cfl=0.5)  # two good steps first
        good = 2
    before = [pb.get_state_stacked(g) for g in range(2)]
    with pytest.raises(FdcgksError) as ei:
        pb.step(nsteps=3, dt=50.0 if how == "huge_dt" else 1e-3)
    assert ei.value.status == ENONPHYS
    assert "non-physical" in str(ei.value)
    after = [pb.get_state_stacked(g) for g in range(2)]
    for g in range(2):
        assert np.array_equal(np.nan_to_num(after[g], nan=7.0), np.nan_to_num(before[g], nan=7.0)), (how, good, g)
