"""The fused stage kernel (interface sweep and update in one kernel marching
up column strips, no interface buffer) against the separate interface sweep,
node sweep and update (GPU).  Both evaluate every quantity with the same
expressions, so stages and steps are compared bit for bit: ragged strips and
row chunks (a chunk may be a single row), every reconstruction and flux
option the fused kernel takes, and the 2048^2 shear layer in the
benchmark's launch configuration."""
import numpy as np
import pytest

import workloads as WL
from tests.helpers import gpu_params, settings

pytestmark = pytest.mark.gpu


def _problem(s, P, D, fused, rows=0):
    from paper_2606_17772_amd import Problem
    pb = Problem(gpu_params(s))
    pb.set_state_stacked(0, P)
    pb.set_state_stacked(1, D)
    pb.fuse_stage = fused
    pb.fused_rows = rows
    return pb


CASES = {
    "vortex_40": lambda: (settings(dim=2, nx=40, ny=40, lx=10.0), WL.vortex(40, seed=1)),
    "rough_130x67": lambda: (settings(dim=2, nx=130, ny=67, lx=1.0), WL.random_rough2d(130, 67, seed=4)),
    "smooth_61x5": lambda: (settings(dim=2, nx=61, ny=5, lx=1.0), WL.random_smooth2d(61, 5, seed=3)),
    "riemann_123x33_62": lambda: (settings(dim=2, nx=123, ny=33, lx=1.0, variant="6-2"), WL.riemann2d(123, seed=2)),
    "shear_ns_64": lambda: (settings(dim=2, nx=64, ny=64, lx=1.0, mu=1e-3, prandtl=0.72), WL.shear_layer(64, seed=0)),
    "vortex_70_linear": lambda: (settings(dim=2, nx=70, ny=70, lx=10.0, variant="linear"), WL.vortex(70, seed=2)),
    "rough_66x20_char": lambda: (settings(dim=2, nx=66, ny=20, lx=1.0, recon_vars="characteristic"),
                                 WL.random_rough2d(66, 20, seed=5)),
    "vortex_64_fp32": lambda: (settings(dim=2, nx=64, ny=64, lx=10.0, fp32_flux=True), WL.vortex(64, seed=3)),
    "smooth_80x48_carried": lambda: (settings(dim=2, nx=80, ny=48, lx=1.0, grad_carried=1),
                                     WL.random_smooth2d(80, 48, seed=6)),
}


def _case(name):
    s, pr = CASES[name]()
    P, D = pr.P[:, :s["ny"], :s["nx"]], pr.D[:, :s["ny"], :s["nx"]]
    return s, np.ascontiguousarray(P), np.ascontiguousarray(D)


@pytest.mark.parametrize("rows", [0, 1, 7])
@pytest.mark.parametrize("name", list(CASES))
def test_fused_stages_bitwise(name, rows):
    s, P, D = _case(name)
    a = _problem(s, P, D, False)
    b = _problem(s, P, D, True, rows)
    dt = a.compute_dt(0.4)
    a1, aa = a.debug_stage(1, dt)
    b1, ba = b.debug_stage(1, dt)
    assert np.array_equal(a1, b1), float(np.abs(a1 - b1).max())
    assert np.array_equal(aa, ba), float(np.abs(aa - ba).max())
    a2 = a.debug_stage(2, dt)
    b2 = b.debug_stage(2, dt)
    assert np.array_equal(a2, b2), float(np.abs(a2 - b2).max())


@pytest.mark.parametrize("name", ["vortex_40", "rough_130x67", "shear_ns_64", "rough_66x20_char"])
def test_fused_steps_bitwise(name):
    """CFL steps (the fold of the wave speeds into the next step's dt
    included), captured as graphs and launched separately."""
    s, P, D = _case(name)
    a = _problem(s, P, D, False)
    b = _problem(s, P, D, True)
    c = _problem(s, P, D, True, 5)
    c.graph_steps = 0
    for rep in range(2):
        ta, na = a.step(nsteps=3, cfl=0.4)
        tb, nb = b.step(nsteps=3, cfl=0.4)
        tc, nc = c.step(nsteps=3, cfl=0.4)
        assert na == nb == nc == 3 and ta == tb == tc, (ta, tb, tc)
        A = a.get_state_all()
        assert np.array_equal(A, b.get_state_all()) and np.array_equal(A, c.get_state_all()), rep


def test_fused_full_size_bitwise():
    """Two CFL steps of the 2048^2 shear layer in the benchmark's launch
    configuration, fused against separate."""
    import torch
    from tests.test_gpu_parity2d import _bench_tiles
    n = 2048
    pr = WL.shear_layer(n, seed=0)
    s = settings(dim=2, nx=n, ny=n, lx=1.0, mu=1e-4, prandtl=0.72)
    dev = torch.device("cuda:0")
    S0 = torch.from_numpy(np.stack([pr.P, pr.D])).to(dev)
    out = []
    for fused in (False, True):
        from paper_2606_17772_amd import Problem
        pb = Problem(gpu_params(s))
        _bench_tiles(pb)
        pb.fuse_stage = fused
        pb.set_state_all(S0)
        t, k = pb.step(nsteps=2, cfl=0.5)
        out.append((t, k, pb.get_state_all(device=dev)))
        del pb
    assert out[0][:2] == out[1][:2]
    assert torch.equal(out[0][2], out[1][2]), float((out[0][2] - out[1][2]).abs().max())


def test_fused_option_rejected_where_it_does_not_apply():
    """Bounded problems and the order-8 flux keep the separate kernels (the
    option is accepted but has no effect), so results stay those of the
    separate path."""
    from tests import test_gpu_boundaries as TB
    s, P, D = TB._case_mixed()
    a = _problem(s, P, D, False)
    b = _problem(s, P, D, True)
    a.step(nsteps=2, cfl=0.4)
    b.step(nsteps=2, cfl=0.4)
    for g in (0, 1):
        assert np.array_equal(a.get_state_stacked(g), b.get_state_stacked(g))


def test_automatic_stage_choice():
    """The default (2) takes the separate sweeps where the fused kernel's row
    chunks would be short (a small grid: the per-kernel timing shows an
    interface sweep) and the fused kernel where they are tall (2048^2: no
    separate interface sweep); 1 forces the fused kernel; other values are
    rejected."""
    from paper_2606_17772_amd import Problem
    s, pr = CASES["vortex_40"]()
    pb = _problem(s, pr.P, pr.D, 2)
    assert pb.fuse_stage == 2
    _, _, kms = pb.step_timed(nsteps=1, cfl=0.5)
    assert kms["edge1"] > 0.0
    pb.fuse_stage = 1
    _, _, kms = pb.step_timed(nsteps=1, cfl=0.5)
    assert kms["edge1"] == 0.0 and kms["update1"] > 0.0
    with pytest.raises(RuntimeError):
        pb.fuse_stage = 3
    n = 2048
    big = Problem(gpu_params(settings(dim=2, nx=n, ny=n, lx=1.0)))
    big.set_state_stacked(0, np.stack([np.ones((n, n)), np.zeros((n, n)), np.zeros((n, n)), 2.5 * np.ones((n, n))] +
                                      [np.zeros((n, n))] * 8))
    big.set_state_stacked(1, np.stack([np.ones((n, n)), np.zeros((n, n)), np.zeros((n, n)), 2.5 * np.ones((n, n))] +
                                      [np.zeros((n, n))] * 8))
    _, _, kms = big.step_timed(nsteps=1, cfl=0.5)
    assert kms["edge1"] == 0.0 and kms["update1"] > 0.0
