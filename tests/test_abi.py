"""The C-ABI library loads and exports every symbol include/*.h declares;
argument validation happens before any device work (CPU only)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    out = set()
    for name in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if name.endswith(".h"):
            src = open(os.path.join(ROOT, "include", name)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            out |= set(re.findall(r"\b(fdcgks(?:3d)?_[a-z_0-9]+)\s*\(", src))
    return sorted(out)


def test_header_declares_the_boundary():
    syms = header_symbols()
    for s in ("fdcgks_create", "fdcgks_set_state", "fdcgks_get_state", "fdcgks_step", "fdcgks_compute_dt",
              "fdcgks_destroy", "fdcgks_last_error", "fdcgks_default_params"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2606_17772_amd import _lib
    L = _lib.load()
    for s in header_symbols():
        assert hasattr(L, s), s
    assert set(header_symbols()) <= set(_lib.SIGNATURES), "binding must declare every ABI symbol"


@pytest.mark.parametrize("cname,pyname", [("fdcgks_params", "Params"), ("fdcgks3d_params", "Params3D")])
def test_params_struct_matches_header(tmp_path, cname, pyname):
    """The binding's params mirrors have the headers' sizes and field offsets
    (a C program compiled against include/ prints them)."""
    import subprocess

    import paper_2606_17772_amd as P
    Params = getattr(P, pyname)
    names = [f[0] for f in Params._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"fdcgks3d.h\"\nint main(void) {\n"
                   f'  printf("%zu\\n", sizeof({cname}));\n'
                   + "".join(f'  printf("%zu\\n", offsetof({cname}, {n}));\n' for n in names)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert vals[0] == C.sizeof(Params)
    assert vals[1:] == [getattr(Params, n).offset for n in names]


def test_defaults():
    from paper_2606_17772_amd import default_params
    p = default_params()
    assert (p.dim, p.nx, p.ny, p.geno_r) == (2, 64, 64, 3)
    assert p.geno_C == 20.0 and p.geno_eps == 1e-15 and p.geno_eps_a == 1e-6
    assert p.geno_d_central == 8.0 and p.geno_d_side == 1.0 and p.gamma == 1.4
    assert p.flux_order == 6


@pytest.mark.parametrize("bad", [
    dict(dim=3), dict(nx=3), dict(ny=2), dict(gamma=1.0), dict(gamma=1.7), dict(mu=-1.0),
    dict(mu=1e-3, prandtl=0.0), dict(flux_variant=7), dict(flux_precision=5), dict(geno_r=0),
    dict(geno_eps=0.0), dict(tau_c1=-1.0), dict(bc=4), dict(bc=-1), dict(lx=0.0), dict(ly=2.0),
    dict(recon_vars=2), dict(dim=1, nx=100, ny=2), dict(grad_update=3), dict(dim=1, nx=100, ny=1, bc=3),
    dict(side=(0, 2, -1, -1)), dict(side=(-1, -1, 1, 0)), dict(side=(5, 5, -1, -1)), dict(bc=2, side=(0, -1, -1, -1)),
    dict(flux_order=7), dict(flux_order=0),
])
def test_create_rejects_bad_params(bad):
    from paper_2606_17772_amd import _lib, default_params
    L = _lib.load()
    p = default_params()
    for k, v in bad.items():
        if k == "side":
            p.side[:] = v
        else:
            setattr(p, k, v)
    h = C.c_void_p()
    st = L.fdcgks_create(C.byref(p), None, C.byref(h))
    assert st == _lib.EINVAL
    assert not h.value
    assert L.fdcgks_last_error(None)


def test_null_arguments():
    from paper_2606_17772_amd import _lib
    L = _lib.load()
    assert L.fdcgks_create(None, None, None) == _lib.EINVAL
    assert L.fdcgks_destroy(None) == _lib.OK
    t = C.c_double(0)
    assert L.fdcgks_step(None, 0.1, 0.5, 1, 0.0, C.byref(t), None) == _lib.EINVAL
    assert L.fdcgks_set_state(None, 0, None, None, None, 0, 0) == _lib.EINVAL
    assert L.fdcgks_get_state(None, 0, None, None, None, 0, 0) == _lib.EINVAL
    assert L.fdcgks_set_state_from_samples(None, None, 0) == _lib.EINVAL
    assert L.fdcgks_diagnostics(None, None) == _lib.EINVAL
    assert L.fdcgks_step_vjp(None, 0.1, None, None, 0) == _lib.EINVAL
    assert L.fdcgks_batch_step(None, 0.5, 1, None, None, None) == _lib.EINVAL
    v = C.c_int64()
    assert L.fdcgks_set_option(None, 0, 1) == _lib.EINVAL
    assert L.fdcgks_get_option(None, 0, C.byref(v)) == _lib.EINVAL
    assert L.fdcgks_autotune(None, 3) == _lib.EINVAL


def test_defaults_3d():
    from paper_2606_17772_amd import make_params3d
    p = make_params3d()
    assert (p.nx, p.ny, p.nz, p.geno_r, p.flux_order) == (32, 32, 32, 3, 6)
    assert p.geno_C == 20.0 and p.gamma == 1.4 and p.lx == 1.0 and p.recon_vars == 0


@pytest.mark.parametrize("bad", [
    dict(nx=3), dict(nz=2), dict(gamma=1.0), dict(gamma=1.7), dict(mu=-1.0), dict(mu=1e-3, prandtl=0.0),
    dict(flux_variant=3), dict(flux_order=7), dict(geno_r=9), dict(geno_eps=0.0), dict(tau_c2=-1.0),
    dict(lx=0.0), dict(grad_update=2), dict(recon_vars=2), dict(nx=1024, ny=1024, nz=128),
])
def test_create3d_rejects_bad_params(bad):
    from paper_2606_17772_amd import _lib, make_params3d
    L = _lib.load()
    p = make_params3d(**bad)
    h = C.c_void_p()
    st = L.fdcgks3d_create(C.byref(p), None, C.byref(h))
    assert st == _lib.EINVAL and not h.value
    assert L.fdcgks3d_last_error(None)
