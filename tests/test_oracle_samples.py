"""Pins of the oracle's state-from-samples construction (Eq.
define-averaged-gradient, D31) against closed forms (CPU): for a periodic
sine field the Gauss difference over one mesh is (2/h) sin(pi h/L) times the
cosine at the node, and the nodal value is the field at the node position
(primary nodes at (i+1/2)h, dual nodes at (i+1)h)."""
import math

import numpy as np

from tests.helpers import oracle_par, settings


def test_samples_2d_closed_form(oracle):
    nx, ny, L = 12, 8, 1.0
    h = L / nx
    Ly = ny * h
    rng = np.random.default_rng(0)
    ph = rng.uniform(0, 2 * math.pi, size=(4, 2))
    kx = np.arange(2 * nx)
    ky = np.arange(2 * ny)
    X = (kx[None, :] + 1) * h / 2
    Y = (ky[:, None] + 1) * h / 2
    S = np.stack([1.0 + 0.1 * np.sin(2 * math.pi * X / L + ph[c, 0]) * np.cos(2 * math.pi * Y / Ly + ph[c, 1])
                  for c in range(4)])
    par = oracle_par(oracle, settings(dim=2, nx=nx, ny=ny, lx=L))
    P, D = oracle.state_from_samples(par, S)
    for g, A in enumerate((P, D)):
        off = 0.5 if g == 0 else 1.0
        x = (np.arange(nx)[None, :] + off) * h
        y = (np.arange(ny)[:, None] + off) * h
        for c in range(4):
            ax, ay = 2 * math.pi * x / L + ph[c, 0], 2 * math.pi * y / Ly + ph[c, 1]
            val = 1.0 + 0.1 * np.sin(ax) * np.cos(ay)
            dx = 0.1 * (2 / h) * math.sin(math.pi * h / L) * np.cos(ax) * np.cos(ay)
            dy = -0.1 * (2 / h) * math.sin(math.pi * h / Ly) * np.sin(ax) * np.sin(ay)
            assert np.abs(A[c] - val).max() < 1e-14
            assert np.abs(A[4 + c] - dx).max() < 1e-12
            assert np.abs(A[8 + c] - dy).max() < 1e-12


def test_samples_1d_closed_form(oracle):
    N, L = 20, 2.0
    h = L / N
    k = np.arange(2 * N)
    X = (k + 1) * h / 2
    S = np.stack([1.0 + 0.2 * np.sin(math.pi * X + c) for c in range(3)])
    par = oracle_par(oracle, settings(dim=1, nx=N, lx=L, dual_1d=1))
    A = oracle.state_from_samples(par, S)
    assert A.shape == (2, 6, N)
    for ln, off in ((0, 0.5), (1, 1.0)):
        x = (np.arange(N) + off) * h
        for c in range(3):
            assert np.abs(A[ln, c] - (1.0 + 0.2 * np.sin(math.pi * x + c))).max() < 1e-14
            d = 0.2 * (2 / h) * math.sin(math.pi * h / 2) * np.cos(math.pi * x + c)
            assert np.abs(A[ln, 3 + c] - d).max() < 1e-12
