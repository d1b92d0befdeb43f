"""Shared test helpers: parameter mapping and error measures (no method
arithmetic)."""
import numpy as np

DEFAULTS = dict(gamma=1.4, mu=0.0, prandtl=1.0, variant="6-4", geno_C=20.0, geno_r=3, geno_eps=1e-15,
                geno_eps_a=1e-6, d_central=8.0, d_side=1.0, tau_c1=0.0, tau_c2=1.0, bc="periodic")

# max-relative parity bar for FP64 (per plane: max |gpu - oracle| / max |oracle|)
TOL = 1e-12


def settings(**kw):
    s = dict(DEFAULTS)
    s.update(kw)
    return s


def oracle_par(O, s):
    return O.make_par(**s)


def gpu_params(s):
    from paper_2606_17772_amd import make_params
    kw = dict(dim=s["dim"], nx=s["nx"], ny=s.get("ny", 1), lx=s["lx"], gamma=s["gamma"], mu=s["mu"],
              prandtl=s["prandtl"], variant=s["variant"], geno_C=s["geno_C"], geno_r=s["geno_r"],
              geno_eps=s["geno_eps"], geno_eps_a=s["geno_eps_a"], geno_d_central=s["d_central"],
              geno_d_side=s["d_side"], tau_c1=s["tau_c1"], tau_c2=s["tau_c2"], bc=s["bc"],
              fp32_flux=s.get("fp32_flux", False), grad_carried=s.get("grad_carried", 0),
              recon_vars=s.get("recon_vars", "conservative"), flux_order=s.get("flux_order", 6))
    if s.get("sides") is not None:
        kw["sides"] = s["sides"]
    if s["dim"] == 2:
        kw["ly"] = s.get("ly", s["lx"] * s["ny"] / s["nx"])
    else:
        kw["dual_1d"] = s.get("dual_1d", 0)
    return make_params(**kw)


def maxrel(g, o, floor=1e-6, axes=None):
    """Largest per-plane relative error; planes are the leading axes up to the
    last two (2D) / last one (1D)."""
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    assert g.shape == o.shape, (g.shape, o.shape)
    if axes is None:
        axes = (-2, -1) if g.ndim >= 3 else (-1,)
    num = np.abs(g - o).max(axis=axes)
    den = np.maximum(np.abs(o).max(axis=axes), floor)
    return float((num / den).max())


def worst_plane(g, o, floor=1e-6):
    num = np.abs(g - o).max(axis=(-2, -1))
    den = np.maximum(np.abs(o).max(axis=(-2, -1)), floor)
    r = num / den
    return np.unravel_index(np.argmax(r), r.shape), float(r.max())


# ------------------------------------------------------------------ scales
# A plane whose exact values vanish (e.g. rho_t of a shear layer) has no
# meaningful relative error; its denominator is floored by the dimensional
# reference scale of the field: rho0, rho0 a, rho0 a^2 for rho, momentum,
# energy (a = largest wave speed |u| + c), divided by the domain length L for
# spatial derivatives, times a/L for time derivatives.
def ref_scales(states, gamma, L, dim=2):
    rho = U = V = None
    rmax, amax = 0.0, 0.0
    for S in states:
        W = np.asarray(S)[: dim + 2]
        rho = W[0]
        U = W[1] / rho
        V = W[2] / rho if dim == 2 else 0.0 * U
        p = (gamma - 1.0) * (W[dim + 1] - 0.5 * rho * (U * U + V * V))
        c = np.sqrt(gamma * p / rho)
        rmax = max(rmax, float(rho.max()))
        amax = max(amax, float((np.maximum(abs(U), abs(V)) + c).max()))
    Wr = [rmax] + [rmax * amax] * dim + [rmax * amax * amax]
    Wr = np.array(Wr)
    return {"W": Wr, "grad": Wr / L, "flux": Wr * amax, "flux_t": Wr * amax * amax / L, "Wt": Wr * amax / L}


def floors_state(sc, dim=2):
    return np.concatenate([sc["W"], sc["grad"], sc["grad"]] if dim == 2 else [sc["W"], sc["grad"]])


def floors_edge(sc):
    one = np.concatenate([sc["flux"], sc["flux_t"], [1.0], sc["W"], sc["W"], sc["Wt"], sc["Wt"]])
    return np.stack([one, one])  # (2 normals, 25)


def floors_node(sc):
    return np.concatenate([sc["flux"], sc["flux_t"], sc["flux"], sc["flux_t"]])


def relerr(g, o, floors, ndim_plane=2):
    """Largest per-plane max|g-o| / max(max|o|, floor); floors broadcast over
    the plane index axes."""
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    assert g.shape == o.shape, (g.shape, o.shape)
    axes = tuple(range(-ndim_plane, 0))
    num = np.abs(g - o).max(axis=axes)
    den = np.maximum(np.abs(o).max(axis=axes), floors)
    r = num / den
    return float(r.max()), np.unravel_index(int(np.argmax(r)), r.shape)


def ulp_sensitivity(run, P, D, floors, trials=2, seed=0):
    """Largest relative change of the oracle's own output when its input is
    perturbed by one ulp (random signs).  Over several steps near
    discontinuities the nonlinear GENO weights amplify round-off, so two
    correct FP64 implementations can only agree to about this level."""
    rng = np.random.default_rng(seed)
    a = run(P, D)
    worst = 0.0
    for _ in range(trials):
        eps = np.finfo(np.float64).eps * rng.choice([-1.0, 1.0], size=P.shape)
        epd = np.finfo(np.float64).eps * rng.choice([-1.0, 1.0], size=D.shape)
        b = run(P * (1 + eps), D * (1 + epd))
        worst = max(worst, relerr(b[0], a[0], floors)[0], relerr(b[1], a[1], floors)[0])
    return worst


CHI = 8  # field of the path function in the interface intermediates (per normal)


def check_edge_intermediates(oracle, par, dt, P, D, gpu, ref, floors, label="", trials=2):
    """Interface intermediates (X, Y families) against the oracle.  Every
    plane is held to 1e-12 except the path function chi itself: chi is a
    ratio of differences of smoothness indicators, which on smooth data are
    differences of nearly equal values, so its round-off is amplified (the
    oracle's own chi moves by up to ~1e-7 under a one-ulp input change on
    smooth cases).  Two implementations that round the indicators
    differently agree on chi only to that level, so chi is held to
    max(1e-12, 4 x the oracle's one-ulp sensitivity of that plane); the
    fluxes it weights are held to 1e-12 like everything else."""
    rng = np.random.default_rng(0)
    sens = [0.0, 0.0]
    for _ in range(trials):
        e1 = np.finfo(np.float64).eps * rng.choice([-1.0, 1.0], size=P.shape)
        e2 = np.finfo(np.float64).eps * rng.choice([-1.0, 1.0], size=D.shape)
        pert = oracle.intermediates2d(par, dt, P * (1 + e1), D * (1 + e2))[:2]
        for f in range(2):
            sens[f] = max(sens[f], float(_plane_rel(pert[f], ref[f], floors)[..., CHI].max()))
    for f, lab in enumerate(("X", "Y")):
        e = _plane_rel(gpu[f], ref[f], floors)
        chi_err = float(e[..., CHI].max())
        print(f"{label} {lab}: chi gpu-oracle {chi_err:.2e}, oracle one-ulp sensitivity {sens[f]:.2e}")
        assert chi_err <= max(TOL, 4 * sens[f]), (lab, chi_err, sens[f])
        e[..., CHI] = 0.0
        assert e.max() <= TOL, (lab, np.unravel_index(int(np.argmax(e)), e.shape), float(e.max()))


def _plane_rel(g, o, fl):
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    num = np.abs(g - o).max(axis=(-2, -1))
    return num / np.maximum(np.abs(o).max(axis=(-2, -1)), fl)


def _ulp_perturbed(rng, a):
    """a with every element moved by one ulp (random signs)."""
    eps = np.finfo(np.float64).eps
    return a * np.where(rng.integers(0, 2, size=a.shape, dtype=np.int8) != 0, 1.0 + eps, 1.0 - eps)


def _sampled_sensitivity(run, arrays, base, floors, trials=2, seed=1):
    """Per-plane largest relative change of the oracle's sampled stage output
    (and stage-1 accumulators) when every input element moves by one ulp."""
    rng = np.random.default_rng(seed)
    worst = np.zeros(base[0].shape[1])
    for _ in range(trials):
        out = run(*[_ulp_perturbed(rng, a) for a in arrays])
        for o, b in zip(out, base):
            for f in range(b.shape[1]):
                d = np.abs(o[:, f] - b[:, f]).max() / max(np.abs(b[:, f]).max(), floors[f])
                worst[f] = max(worst[f], d)
    return worst


def check_full_size_sampled(oracle, s, P, D, pb, ns=48, seed=0, label=""):
    """Both stages of one step at full size on sampled nodes of both grids
    (corner and edge nodes included), against the oracle's sampled stage.

    Every plane (values, averaged gradients, the stage-1 accumulators) is held
    to max(1e-12, 4 x the oracle's own one-ulp sensitivity of that plane at
    the same sampled nodes), measured here by running the oracle's stage again
    on inputs moved by one ulp.  Relative errors use the dimensional floors of
    ref_scales (|W|/L for gradients).  The averaged gradient is the Gauss
    difference of two O(|W|) interface values divided by h (Eq.
    define-averaged-gradient), so its round-off grows like n eps relative to
    |W|/L; the measured sensitivity carries that growth, nothing else widens
    the bar.  Stage 2 starts from the GPU's own stage-1 buffers; its
    sensitivity is measured on those inputs."""
    dt = pb.compute_dt(0.5)
    par = oracle.make_par(**s)
    rng = np.random.default_rng(seed)
    grid = rng.integers(0, 2, ns)
    shapes = [P.shape[1:], D.shape[1:]]
    corners = [(0, 0), (0, 1), (1, 0), (1, 1)]
    jj = np.array([(shapes[g][0] - 1) * corners[k][0] if k < 4 else rng.integers(0, shapes[g][0])
                   for k, g in enumerate(grid)])
    ii = np.array([(shapes[g][1] - 1) * corners[k][1] if k < 4 else rng.integers(0, shapes[g][1])
                   for k, g in enumerate(grid)])
    sc = ref_scales([P, D], s["gamma"], s["lx"])
    fl = floors_state(sc)

    def rel(g, o):
        return np.array([np.abs(g[:, f] - o[:, f]).max() / max(np.abs(o[:, f]).max(), fl[f])
                         for f in range(o.shape[1])])

    def judge(stage, errs, sens):
        bar = np.maximum(TOL, 4.0 * sens)
        print(f"{label} stage {stage}: max-relative error {errs.max():.2e} (values {errs[:4].max():.2e}, "
              f"gradients {errs[4:].max():.2e}); oracle one-ulp sensitivity {sens.max():.2e}; "
              f"bar {bar.max():.2e}", flush=True)
        assert (errs <= bar).all(), (stage, errs, bar)

    run1 = lambda A, B: oracle.stage2d_sample(par, 1, dt, A, B, grid, jj, ii)  # noqa: E731
    o1, a1 = run1(P, D)
    g1, ga = pb.debug_stage(1, dt)
    gs = np.stack([g1[grid[k]][:, jj[k], ii[k]] for k in range(ns)])
    gas = np.stack([ga[grid[k]][:, jj[k], ii[k]] for k in range(ns)])
    sens1 = _sampled_sensitivity(run1, [P, D], (o1, a1), fl)
    judge(1, np.maximum(rel(gs, o1), rel(gas, a1)), sens1)

    A0, A1 = np.ascontiguousarray(g1[0]), np.ascontiguousarray(g1[1])
    C0, C1 = np.ascontiguousarray(ga[0]), np.ascontiguousarray(ga[1])
    run2 = lambda A, B, X, Y: oracle.stage2d_sample(par, 2, dt, A, B, grid, jj, ii, accP=X, accD=Y)[:1]  # noqa: E731
    (o2,) = run2(A0, A1, C0, C1)
    g2 = pb.debug_stage(2, dt)
    gs2 = np.stack([g2[grid[k]][:, jj[k], ii[k]] for k in range(ns)])
    sens2 = _sampled_sensitivity(run2, [A0, A1, C0, C1], (o2,), fl)
    judge(2, rel(gs2, o2), sens2)
