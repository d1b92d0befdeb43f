"""Launch machinery (GPU): captured-step replay and launch shapes change the
schedule, never the arithmetic, so every comparison here is bitwise."""
import numpy as np
import pytest

import workloads as WL
from tests.helpers import gpu_params, settings

pytestmark = pytest.mark.gpu


def _problem(s, pr, **opt):
    from paper_2606_17772_amd import Problem
    pb = Problem(gpu_params(s))
    pb.set_state_all(np.ascontiguousarray(np.stack([pr.P, pr.D])))
    for k, v in opt.items():
        setattr(pb, k, v)
    return pb


def _cases():
    return [
        (settings(dim=2, nx=70, ny=37, lx=1.0), WL.random_smooth2d(70, 37, seed=3)),
        (settings(dim=2, nx=36, ny=36, lx=1.0, mu=1e-3, prandtl=0.72), WL.shear_layer(36, seed=2, k=20.0)),
    ]


@pytest.mark.parametrize("case,k", [(0, 1), (1, 1), (0, 2), (1, 3)])
def test_graph_replays_match_separate_launches(case, k):
    """Several replays of the captured steps (k steps per graph, remainders
    launched separately), with eager work (state reads) and synchronisations
    between them, each checked against the same steps launched kernel by
    kernel."""
    s, pr = _cases()[case]
    a = _problem(s, pr, graph_steps=k)
    b = _problem(s, pr, use_graph=False)
    assert a.graph_steps == k and not b.use_graph
    ta = tb = 0.0
    for rep in range(4):
        ta, na = a.step(nsteps=1 + rep, cfl=0.5, t=ta)
        tb, nb = b.step(nsteps=1 + rep, cfl=0.5, t=tb)
        assert na == nb == 1 + rep and ta == tb
        assert np.array_equal(a.get_state_all(), b.get_state_all()), rep
    # fixed dt (other graph key) and a t_end inside the run
    ta, na = a.step(nsteps=50, dt=1e-3, t_end=ta + 3.5e-3, t=ta)
    tb, nb = b.step(nsteps=50, dt=1e-3, t_end=tb + 3.5e-3, t=tb)
    assert na == nb == 4 and ta == tb
    assert np.array_equal(a.get_state_all(), b.get_state_all())


def test_every_launch_shape_gives_identical_results():
    s, pr = _cases()[0]
    ref = _problem(s, pr)
    assert ref.tiles() == {"edge": (64, 2), "node": (64, 1), "update": (128, 1)}
    ref.step(nsteps=2, cfl=0.5)
    want = ref.get_state_all()
    shapes = [(64, 4), (64, 2), (128, 2), (32, 8), (256, 1), (128, 1), (64, 1), (32, 4)]
    for kernel in ("edge", "node", "update"):
        for x, y in shapes:
            if kernel == "edge" and y % 2:
                continue
            pb = _problem(s, pr)
            pb.set_tile(kernel, x, y)
            assert pb.tiles()[kernel] == (x, y)
            pb.step(nsteps=2, cfl=0.5)
            assert np.array_equal(pb.get_state_all(), want), (kernel, x, y)


@pytest.mark.parametrize("case", [0, 1])
def test_fused_node_sweep_is_bitwise_equal(case):
    """Nodal fluxes evaluated inside the update kernel (tile plus halo in
    LDS) against the separate node sweep through the node buffer, several
    steps, with the graphs on."""
    s, pr = _cases()[case]
    a = _problem(s, pr)
    b = _problem(s, pr)
    a.fuse_stage = b.fuse_stage = False  # the stage fusion takes precedence over the node fusion
    b.fuse_nodes = True
    assert b.fuse_nodes and not a.fuse_nodes
    for rep in range(3):
        ta, na = a.step(nsteps=2, cfl=0.5)
        tb, nb = b.step(nsteps=2, cfl=0.5)
        assert na == nb == 2 and ta == tb
        assert np.array_equal(a.get_state_all(), b.get_state_all()), rep


@pytest.mark.parametrize("case", [0, 1, "walled"])
def test_cfl_fold_matches_fresh_reduction(case):
    """Within one call, the time step of every CFL step after the first comes
    from the wave speeds the previous step's stage-2 update folded; one step
    per call reduces them from the stored state.  Both give the same time
    steps and states bit for bit, with and without captured steps."""
    from paper_2606_17772_amd import Problem
    from tests import test_gpu_boundaries as TB
    if case == "walled":  # the dual grid holds one more node per bounded axis
        s, P, D = TB._case_mixed()
    else:
        s, pr = _cases()[case]
        P, D = pr.P, pr.D

    def make(**opt):
        pb = Problem(gpu_params(s))
        pb.set_state_stacked(0, P)
        pb.set_state_stacked(1, D)
        for k, v in opt.items():
            setattr(pb, k, v)
        return pb

    one, run, cap = make(use_graph=False), make(use_graph=False), make(graph_steps=3)
    t1 = 0.0
    for _ in range(7):
        t1, n = one.step(nsteps=1, cfl=0.5, t=t1)
        assert n == 1
    for pb in (run, cap):
        t, n = pb.step(nsteps=7, cfl=0.5)
        assert n == 7 and t == t1
        for g in (0, 1):
            assert np.array_equal(pb.get_state_stacked(g), one.get_state_stacked(g))


def test_invalid_launch_shapes_rejected():
    from paper_2606_17772_amd import FdcgksError
    s, pr = _cases()[0]
    pb = _problem(s, pr)
    for kernel, x, y in (("edge", 64, 1), ("edge", 64, 3), ("node", 48, 4), ("update", 64, 8), ("node", 32, 1)):
        with pytest.raises(FdcgksError) as ei:
            pb.set_tile(kernel, x, y)
        assert ei.value.status == -1
    assert pb.tiles()["edge"] == (64, 2)


def test_autotune_keeps_results():
    pr = WL.vortex(128, seed=1)
    s = settings(dim=2, nx=128, ny=128, lx=10.0)
    a = _problem(s, pr)
    tiles = a.autotune(reps=3)
    assert set(tiles) == {"edge", "node", "update"}
    ex, ey = tiles["edge"]
    assert ex * ey <= 256 and ey % 2 == 0
    assert np.array_equal(a.get_state_all(), np.stack([pr.P, pr.D]))  # the state was not advanced
    b = _problem(s, pr)
    a.step(nsteps=3, cfl=0.5)
    b.step(nsteps=3, cfl=0.5)
    assert np.array_equal(a.get_state_all(), b.get_state_all())
    print("autotuned shapes at 128^2:", tiles)
