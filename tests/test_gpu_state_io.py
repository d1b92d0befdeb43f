"""State input and output at the C boundary (GPU): the state built on the
device from point samples equals the oracle's construction bit for bit (the
same divisions), and padded-row (strided) copies in and out equal dense
ones.  A step from the sampled state then matches the oracle at the usual
bar."""
import math

import numpy as np
import pytest

import workloads as WL
from tests.helpers import TOL, floors_state, gpu_params, oracle_par, ref_scales, relerr, settings

pytestmark = pytest.mark.gpu


def _samples2d(nx, ny, L=1.0, seed=0):
    h = L / nx
    Ly = ny * h
    rng = np.random.default_rng(seed)
    X = (np.arange(2 * nx)[None, :] + 1) * h / 2
    Y = (np.arange(2 * ny)[:, None] + 1) * h / 2
    a, b = rng.uniform(0, 2 * math.pi, 2)
    rho = 1.0 + 0.2 * np.sin(2 * math.pi * X / L + a) * np.cos(2 * math.pi * Y / Ly + b)
    U = 0.3 + 0.1 * np.cos(2 * math.pi * (X / L + Y / Ly))
    V = -0.2 + 0.1 * np.sin(2 * math.pi * X / L)
    p = 1.0 + 0.1 * np.cos(2 * math.pi * Y / Ly + a)
    return np.ascontiguousarray(WL.conservative(rho, U, V, p))


def test_state_from_samples_2d(oracle):
    nx, ny = 70, 37
    S = _samples2d(nx, ny)
    s = settings(dim=2, nx=nx, ny=ny, lx=1.0)
    par = oracle_par(oracle, s)
    P, D = oracle.state_from_samples(par, S)
    from paper_2606_17772_amd import Problem
    pb = Problem(gpu_params(s))
    pb.set_state_from_samples(S)
    assert np.array_equal(pb.get_state_stacked(0), P)
    assert np.array_equal(pb.get_state_stacked(1), D)
    dt = 0.2 * (1.0 / nx) / 3
    oP, oD, _, _ = oracle.stage2d(par, 1, dt, P, D)
    g1, _ = pb.debug_stage(1, dt)
    fl = floors_state(ref_scales([P, D], s["gamma"], s["lx"]))
    assert relerr(g1[0], oP, fl)[0] <= TOL and relerr(g1[1], oD, fl)[0] <= TOL


def test_state_from_samples_device_array(oracle):
    import torch
    nx, ny = 40, 40
    S = _samples2d(nx, ny, seed=1)
    s = settings(dim=2, nx=nx, ny=ny, lx=1.0)
    P, D = oracle.state_from_samples(oracle_par(oracle, s), S)
    from paper_2606_17772_amd import Problem
    pb = Problem(gpu_params(s))
    pb.set_state_from_samples(torch.from_numpy(S).to("cuda:0"))
    torch.cuda.synchronize()
    assert np.array_equal(pb.get_state_stacked(0), P) and np.array_equal(pb.get_state_stacked(1), D)


def test_state_from_samples_1d(oracle):
    N = 100
    h = 2.0 / N
    x = (np.arange(2 * N) + 1) * h / 2
    S = np.ascontiguousarray(WL.conservative1d(1.0 + 0.2 * np.sin(math.pi * x), 1.0, 1.0))
    s = settings(dim=1, nx=N, lx=2.0, dual_1d=1)
    A = oracle.state_from_samples(oracle_par(oracle, s), S)
    from paper_2606_17772_amd import Problem
    pb = Problem(gpu_params(s))
    pb.set_state_from_samples(S)
    for ln in range(2):
        assert np.array_equal(pb.get_state_stacked(ln).reshape(6, N), A[ln])


def test_state_from_samples_rejects_bounded():
    from paper_2606_17772_amd import FdcgksError, Problem
    s = settings(dim=2, nx=16, ny=16, lx=1.0, bc="reflecting")
    pb = Problem(gpu_params(s))
    with pytest.raises(FdcgksError, match="periodic"):
        pb.set_state_from_samples(np.zeros((4, 32, 32)))


@pytest.mark.parametrize("bounded", [False, True])
def test_strided_copies(bounded):
    from paper_2606_17772_amd import FdcgksError, Problem
    nx, ny = 33, 20
    s = settings(dim=2, nx=nx, ny=ny, lx=1.0, bc="reflecting" if bounded else "periodic")
    pb = Problem(gpu_params(s))
    rng = np.random.default_rng(0)
    stride = nx + 1 + 7
    for g in range(2):
        ny_g, nx_g = pb.grid_dims(g)
        dense = rng.uniform(0.5, 1.5, size=(3, 4, ny_g, nx_g))
        padded = np.full((3, 4, ny_g, stride), -7.0)
        padded[..., :nx_g] = dense
        pb.set_state(g, *(np.ascontiguousarray(padded[f]).ravel() for f in range(3)), row_stride=stride)
        assert np.array_equal(pb.get_state_stacked(g), dense.reshape(12, ny_g, nx_g))
        out = pb.get_state_strided(g, stride)
        for f in range(3):
            o = out[f].reshape(4, ny_g, stride)
            assert np.array_equal(o[..., :nx_g], dense[f])
            assert np.all(o[..., nx_g:] == 0.0)
    with pytest.raises(FdcgksError, match="row_stride"):
        pb.set_state(0, *(np.zeros(4 * ny * nx) for _ in range(3)), row_stride=nx - 1)
