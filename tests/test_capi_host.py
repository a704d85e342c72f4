"""CPU tests of the C ABI library: exported symbols, error paths that need no
device, and the FP64 host plan tables checked against the oracle's dense T."""
import ctypes
import re

import numpy as np
import pytest

from oracle import dsbt as odsbt
from paper_1509_07115_amd import _lib, host_ftb_tables

HEADER = "include/dsbt.h"


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\*\s]+?\b(dsbt_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol(built_lib):
    names = _declared_functions()
    assert len(names) >= 12
    assert sorted(names) == sorted(_lib.EXPORTED)
    lib = ctypes.CDLL(built_lib)
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings_and_host_errors(built_lib):
    lib = _lib.load()
    assert lib.dsbt_status_string(0) == b"ok"
    need = ctypes.c_int64()
    # N not a power of two, l too large, tile below n0: rejected without a device
    assert lib.dsbt_host_ftb_tables(100, 3, 4, None, 0, ctypes.byref(need)) == -2
    assert lib.dsbt_host_ftb_tables(64, 127, 64, None, 0, ctypes.byref(need)) == -2
    assert lib.dsbt_host_ftb_tables(64, 31, 8, None, 0, ctypes.byref(need)) == -2
    assert b"tile" in lib.dsbt_last_error()
    h = ctypes.c_void_p()
    assert lib.dsbt_plan_create(None, None, 0, None, None) == -1
    assert lib.dsbt_plan_create(ctypes.byref(h), None, 0, None, None) in (-1, -7)
    assert lib.dsbt_forward(None, None, None, None) == -1
    assert lib.dsbt_autotune(None, 0, None, 1, None, None, None, None) == -1


def tiled_forward(blocks, f, ell):
    """Run the tile recurrence of the plan in numpy FP64 (the GPU kernel's math)."""
    NT, R, _ = blocks.shape
    k = (ell + 1) // 2
    B = R - k
    p = odsbt.parity_p(ell)
    g = f * odsbt.weights_w(len(f), ell)
    mu = np.zeros(k, dtype=f.dtype)
    b = np.zeros_like(f)
    for J in range(NT):
        out = blocks[J] @ np.concatenate([g[J * B:(J + 1) * B], mu])
        b[J * B:(J + 1) * B] = out[:B]
        mu = out[B:]
    b[:k] = (-1) ** p * mu
    return b


def tiled_inverse(blocks, b, ell):
    NT, R, _ = blocks.shape
    k = (ell + 1) // 2
    B = R - k
    p = odsbt.parity_p(ell)
    lam = (-1) ** p * b[:k].copy()
    h = np.zeros_like(b)
    for J in range(NT - 1, -1, -1):
        out = blocks[J].T @ np.concatenate([b[J * B:(J + 1) * B], lam])
        h[J * B:(J + 1) * B] = out[:B]
        lam = out[B:]
    return h * odsbt.weights_w(len(b), ell)


@pytest.mark.parametrize("N,ell,B", [(16, 0, 4), (16, 1, 4), (16, 2, 4), (32, 7, 8), (64, 13, 8),
                                     (64, 14, 16), (128, 31, 16), (128, 31, 64), (256, 62, 32),
                                     (256, 63, 32), (256, 126, 64), (512, 127, 64), (64, 126, 64)])
def test_host_tables_reproduce_dense_T(built_lib, N, ell, B):
    blocks = host_ftb_tables(N, ell, B)
    T = odsbt.ftb_matrix(N, ell)
    rng = np.random.default_rng(N + ell)
    f = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    assert np.max(np.abs(tiled_forward(blocks, f, ell) - T @ f)) < 1e-12 * np.max(np.abs(T @ f)) * 10
    bb = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    assert np.max(np.abs(tiled_inverse(blocks, bb, ell) - T.T @ bb)) < 1e-11


def test_host_tables_are_independent_of_N(built_lib):
    # rows of T do not depend on N, so the first tiles agree across grid sizes
    a = host_ftb_tables(128, 21, 16)
    b = host_ftb_tables(512, 21, 16)
    assert np.array_equal(a, b[: a.shape[0]])


@pytest.mark.parametrize("N,ell,rmax", [(64, 0, 12.8), (64, 1, 12.8), (64, 2, 12.8), (128, 7, 25.6),
                                        (256, 31, 51.2), (512, 64, 102.4), (1024, 127, 204.8)])
def test_corrected_momenta_match_oracle_roots(built_lib, N, ell, rmax):
    # eq. kcorr: the library's FP64 root scan and bisection against the oracle's
    # scan and Brent refinement of SciPy's spherical_jn
    from oracle import sbf
    from paper_1509_07115_amd import kinetic_momenta
    k = kinetic_momenta(N, ell, rmax, "corrected")
    kx = odsbt.n_extra(ell)
    assert np.all(k[:kx] == N * odsbt.delta_k(rmax))
    ref = sbf.corrected_momenta(N, rmax, ell)
    assert np.max(np.abs(k[kx:] - ref)) < 1e-10 * np.max(ref)
    plain = kinetic_momenta(N, ell, rmax, "plain")
    p = odsbt.parity_p(ell)
    assert np.allclose(plain[kx:], np.arange(kx + p, N + p) * odsbt.delta_k(rmax), rtol=1e-15, atol=0)


def test_plan_opts_layout_matches_the_header(tmp_path):
    # the ctypes mirror of dsbt_plan_opts against the C compiler's layout of
    # the header (sizes and field offsets)
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    fields = [f[0] for f in _lib.PlanOpts._fields_]
    src = tmp_path / "layout.c"
    body = "".join(f'    printf("{f} %zu\\n", offsetof(dsbt_plan_opts, {f}));\n' for f in fields)
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "dsbt.h"\nint main(void) {\n'
                   '    printf("size %zu\\n", sizeof(dsbt_plan_opts));\n' + body + "    return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", "include", str(src), "-o", str(exe)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                       text=True).stdout.splitlines())
    assert int(out["size"]) == ctypes.sizeof(_lib.PlanOpts)
    for f in fields:
        assert int(out[f]) == getattr(_lib.PlanOpts, f).offset, f


def test_plan_opts_validation_without_a_device(built_lib):
    # option checks come before the device lookup: they fail the same way with
    # or without a GPU
    lib = _lib.load()
    ch = (_lib.Channel * 1)(_lib.Channel(64, 3, 6.4, 0))
    h = ctypes.c_void_p()
    o = _lib.PlanOpts()
    o.check_finite = 2
    assert lib.dsbt_plan_create(ctypes.byref(h), ch, 1, ctypes.byref(o), None) == -1
    assert b"check_finite" in lib.dsbt_last_error()
    o = _lib.PlanOpts()
    o.dev_alloc = _lib.ALLOC_FN(lambda n, c: None)    # dev_free missing
    assert lib.dsbt_plan_create(ctypes.byref(h), ch, 1, ctypes.byref(o), None) == -1
    assert b"together" in lib.dsbt_last_error()
    assert lib.dsbt_status_string(_lib.DSBT_ERR_NONFINITE) == b"NaN or infinity in the data"
