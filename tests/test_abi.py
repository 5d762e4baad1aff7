"""The C-ABI library loads and exports every symbol include/lbm.h declares;
host-side argument checks (no GPU work)."""

import ctypes as C
import os
import re

import pytest

from paper_1309_6726_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:lbm|surr)_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_1309_6726_amd import lbm
    if not os.path.exists(lbm.LIB_PATH):
        from paper_1309_6726_amd import build
        build.build()
    return lbm


def test_every_declared_symbol_is_exported(L):
    lib = L.lib()
    names = declared("lbm.h")
    assert "lbm_init" in names and "lbm_step" in names and "lbm_observe" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTS)


def test_workspace_and_param_checks(L):
    p = inputs.config1().params
    n = L.workspace_bytes(p)
    N = 1024 * 64
    assert n >= N * (2 * 18 * 4 + 2 * 5 * 4 + 1 + 8 + 4 + 12 + 16)
    for bad in (dict(tau=0.5), dict(nx=2), dict(k_r=0.3), dict(tau_g=0.4), dict(threshold=0.0),
                dict(k_r=1e-3, tau_g=0.0), dict(W=10, y0=60), dict(x_in=900, x_out=901)):
        with pytest.raises(L.LbmError) as e:
            L.workspace_bytes(p.replace(**bad))
        assert e.value.status == L.LBM_EINVAL
        assert L.lib().lbm_last_error()


def test_size_limit(L):
    """32-bit element offsets: 23 population planes of P = ceil64(nx ny)
    elements must stay below 2^31.  9472 x 9856 (the lattice of the GPU
    maximum-size test) is accepted, three more rows are refused."""
    p = inputs.config1().params.replace(nx=9472, ny=9856, W=0, x_in=0, x_out=0, y0=0)
    P = (p.nx * p.ny + 63) // 64 * 64
    assert 23 * P <= 2**31 - 1 < 23 * (P + 3 * p.nx)
    assert L.workspace_bytes(p) > 0
    with pytest.raises(L.LbmError) as e:
        L.workspace_bytes(p.replace(ny=p.ny + 3))
    assert e.value.status == L.LBM_EINVAL


def test_strerror(L):
    lib = L.lib()
    for s in (0, -1, -2, -3, -4, -5):
        assert lib.lbm_strerror(s)
    assert lib.lbm_strerror(L.LBM_ENONFINITE).decode().startswith("non-finite")


def test_null_arguments_rejected_without_device(L):
    lib = L.lib()
    assert lib.lbm_step(None, 1) == L.LBM_EINVAL
    assert lib.lbm_observe(None, None) == L.LBM_EINVAL
    assert lib.lbm_set_tile(None, 64, 4) == L.LBM_EINVAL
    n = C.c_size_t(0)
    assert lib.lbm_save(None, None, 0, C.byref(n)) == L.LBM_EINVAL
    pp = L.Params.of(inputs.config0().params)
    out = C.c_void_p()
    # NULL inputs and a too-small workspace fail before any device call
    assert lib.lbm_init(C.byref(pp), None, None, None, None, None, None, 0, C.byref(out)) == L.LBM_EINVAL


def test_blob_layout_size(L):
    p = inputs.config1().params
    import numpy as np
    N = p.nx * p.ny
    blob = L.make_blob(p, np.zeros((18, p.ny, p.nx)), np.zeros((p.ny, p.nx), np.uint8))
    assert len(blob) == 40 + 18 * N * 4 + 5 * N * 4 + N + N * 8 + N * 4 + 3 * N * 4
