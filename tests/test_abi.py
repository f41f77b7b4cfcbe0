"""The C ABI without a GPU: the library loads, exports every symbol that
include/ctm.h declares, and rejects invalid arguments before touching a device."""
import ctypes
import os
import re

import pytest

import paper_2112_13184_amd as pkg
from paper_2112_13184_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ctm.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return sorted(set(re.findall(r"\b(ctm_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libctm.so not built (run __graft_entry__.build())")
    return B.load()


def test_header_declares_the_binding_exports():
    assert _declared() == sorted(B.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    raw = ctypes.CDLL(B.LIB_PATH)
    missing = [name for name in _declared() if not hasattr(raw, name)]
    assert not missing, missing


def test_invalid_configs_are_rejected(lib):
    good = dict(Lx=2, Ly=2, D=3, chi=20)
    assert lib.ctm_footprint_bytes(ctypes.byref(B.make_config(**good))) > 0
    bad = [dict(good, Lx=0), dict(good, D=9), dict(good, chi=0), dict(good, layers=3),
           dict(good, rsvd_power_iters=-1), dict(good, svd_rel_cutoff=1.5),
           dict(good, Lx=5, Ly=4)]
    for kw in bad:
        cfg = B.make_config(**kw)
        assert lib.ctm_footprint_bytes(ctypes.byref(cfg)) == 0, kw
        h = ctypes.c_void_p()
        dummy = (ctypes.c_double * 1)()
        st = lib.ctm_init(ctypes.byref(cfg), ctypes.cast(dummy, B._DP), 0, None, ctypes.byref(h))
        assert st == B.CTM_EINVAL and not h.value, kw
        assert lib.ctm_last_error(None)


def test_null_handles(lib):
    assert lib.ctm_move(None, 0) == B.CTM_EINVAL
    assert lib.ctm_sweep(None, 1, 1e-8, None, None, None) == B.CTM_EINVAL
    assert lib.ctm_env_bytes(None) == 0
    assert lib.ctm_init(None, None, 0, None, None) == B.CTM_EINVAL
    assert lib.ctm_last_error(None)
    lib.ctm_free(None)


def test_footprint_grows_with_chi(lib):
    f = [lib.ctm_footprint_bytes(ctypes.byref(B.make_config(2, 2, 6, chi))) for chi in (32, 64, 144)]
    assert 0 < f[0] < f[1] < f[2]
    # the resident environment alone: 4 sites x (4 C + 8 T copies)
    assert f[2] > 8 * 4 * (4 * 144 ** 2 + 8 * 144 ** 2 * 36)


def test_package_reexports_binding():
    assert pkg.Ctm is B.Ctm and callable(pkg.load)


def test_simple_update_rejects_bad_arguments_before_any_device_call(lib):
    def create(Lx, Ly, D, d, batch, gamma, lam):
        cfg = B.ctm_su_config(Lx, Ly, d, D, batch, None)
        h = ctypes.c_void_p()
        g = (ctypes.c_double * max(len(gamma), 1))(*gamma)
        lm = (ctypes.c_double * max(len(lam), 1))(*lam)
        st = lib.ctm_su_create(ctypes.byref(cfg), ctypes.cast(g, B._DP), ctypes.cast(lm, B._DP), ctypes.byref(h))
        return st, h.value
    N, D, d = 4, 2, 2
    gam = [0.5] * (N * D ** 4 * d)
    lam = [1.0] * (N * 2 * D)
    assert create(2, 1, D, d, 1, gam[:32], lam[:8])[0] == B.CTM_EINVAL      # Ly = 1
    assert create(2, 2, 9, d, 1, gam, lam)[0] == B.CTM_EINVAL                # D > 8
    assert create(2, 2, 8, 3, 1, gam, lam)[0] == B.CTM_EINVAL                # core of 72 columns
    assert create(2, 2, D, d, 0, gam, lam)[0] == B.CTM_EINVAL                # empty batch
    bad_w = list(lam)
    bad_w[3] = -0.1
    assert create(2, 2, D, d, 1, gam, bad_w)[0] == B.CTM_EINVAL              # negative weight
    bad_g = list(gam)
    bad_g[7] = float("nan")
    st, h = create(2, 2, D, d, 1, bad_g, lam)
    assert st == B.CTM_EINVAL and not h
    assert lib.ctm_su_last_error(None)
    assert lib.ctm_su_run(None, 1) == B.CTM_EINVAL
    assert lib.ctm_fu_step(None, None, 0.01, 1, 1) == B.CTM_EINVAL
    lib.ctm_su_free(None)
