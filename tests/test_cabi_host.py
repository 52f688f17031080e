"""CPU checks of the C ABI library: it loads, exports every declared entry point,
rejects bad arguments, and its host-built plan tables (Algorithm 1, steps 1-2)
match the oracle's: the (k, q) index tables bit for bit, the FP64 tables to
rounding level.  No compute call is made (no GPU here)."""

import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1412_0781_amd import FBError, Plan
from paper_1412_0781_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "ffbspca.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fb_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = _lib.lib()
    syms = _declared_symbols()
    assert len(syms) >= 16
    for s in syms:
        assert hasattr(lib, s), s
    assert {name for name, _, _ in _lib.SIGNATURES} == set(syms)


def test_error_strings():
    lib = _lib.lib()
    for code in [0, -1, -2, -3, -4, -5, -6, -7]:
        assert lib.fb_error_string(code)
    assert lib.fb_error_string(-1) == b"invalid argument"


@pytest.mark.parametrize("L,c,R", [(32, 0.6, 16), (32, 0.0, 16), (32, 0.5, 17), (1, 0.5, 0.5), (4, 0.5, 0.5)])
def test_invalid_plan_arguments(L, c, R):
    with pytest.raises(FBError):
        Plan(L, c, R, device=False)


def test_host_plan_rejects_compute_without_device():
    p = Plan(16, 0.5, 8, device=False)
    lib = _lib.lib()
    # a compute call on a host-only plan returns FB_ERR_NO_DEVICE before touching any pointer
    assert lib.fb_expand(p._h, 1, 1, 1, 0, 1, 1 << 20, None) == -5
    assert lib.fb_expand(p._h, 1, -1, 1, 0, 1, 1 << 20, None) == -1       # n < 0
    assert lib.fb_expand(p._h, 1, 1, 1, 7, 1, 1 << 20, None) == -1        # bad precision
    assert lib.fb_expand(p._h, None, 0, None, 0, None, 0, None) == 0      # n = 0 is a no-op
    assert lib.fb_eig(p._h, 1, 1, None, 0, 1, 1, None, None, 1, 1 << 20, None) == -1   # count <= 0
    assert lib.fb_expand_weighted(p._h, 1, 1, 1, 0, 2, 1, 1 << 20, None) == -1       # bad weight mode
    assert lib.fb_expand_weighted(p._h, 1, 1, 1, 0, 0, 1, 1 << 20, None) == -5
    cnt = ctypes.c_int64(0)
    assert lib.fb_covariance(p._h, 1, 1, 1, 1, None, None, ctypes.byref(cnt), 0, 8, 1 << 20, None) == -5
    # the CTF envelope: argument checks, then the host-only plan
    assert lib.fb_ctf_filter(p._h, 1.0, 0.0197, 2.5e4, 0.1, 100.0, None, None) == -1        # no output
    assert lib.fb_ctf_filter(p._h, 0.0, 0.0197, 2.5e4, 0.1, 100.0, 1, None) == -1           # pixel size
    assert lib.fb_ctf_filter(p._h, 1.0, float("nan"), 2.5e4, 0.1, 100.0, 1, None) == -1     # non-finite
    assert lib.fb_ctf_filter(p._h, 1.0, 0.0197, 2.5e4, 0.1, 100.0, 1, None) == -5
    cnt.value = -1
    assert lib.fb_covariance(p._h, 1, 1, 1, 1, None, None, ctypes.byref(cnt), 0, 8, 1 << 20, None) == -1
    # the imaginary parts need a second set of per-run partial sums
    assert lib.fb_covariance_workspace_bytes(p._h, 5000, 1) > lib.fb_covariance_workspace_bytes(p._h, 5000, 0) > 0


CONFIGS = [(8, 0.5, 4), (15, 0.5, 7.5), (32, 0.5, 16), (42, 1 / 3, 21), (121, 1 / 3, 60), (128, 0.5, 64),
           (240, 0.196, 98), (256, 0.5, 128), (360, 0.5, 180)]


@pytest.mark.parametrize("L,c,R", CONFIGS)
def test_index_tables_bit_exact(L, c, R):
    po = oracle.plan(L, c, R)
    pg = Plan(L, c, R, device=False)
    assert (pg.n_xi, pg.n_theta, pg.k_max, pg.p0) == (po.n_xi, po.n_theta, po.k_max, po.p[0])
    assert pg.p_half == po.p_half and pg.p_total == po.p_total
    assert np.array_equal(pg.p, np.array(po.p))
    assert np.array_equal(pg.coef_off, po.coef_off)
    assert np.array_equal(pg.k, po.kq[:, 0]) and np.array_equal(pg.q, po.kq[:, 1])
    cov = np.zeros(po.k_max + 2, np.int64)
    cov[1:] = np.cumsum(np.array(po.p) ** 2)
    assert np.array_equal(pg.cov_off, cov)


@pytest.mark.parametrize("L,c,R", [(32, 0.5, 16), (42, 1 / 3, 21), (64, 0.5, 32)])
def test_fp64_tables_match_oracle(L, c, R):
    po = oracle.plan(L, c, R)
    pg = Plan(L, c, R, device=False)
    roots, norms, xi, w, radial = pg.host_tables()
    ro = np.concatenate(po.roots)
    no = np.concatenate(po.norms)
    assert np.max(np.abs(roots - ro) / ro) < 1e-14
    assert np.max(np.abs(norms - no) / no) < 1e-12
    assert np.max(np.abs(xi - po.xi)) < 1e-15 and np.max(np.abs(w - po.w)) < 1e-15
    Bo = np.concatenate(po.B, axis=0)
    assert np.max(np.abs(radial - Bo)) < 1e-12 * np.max(np.abs(Bo))


def test_odd_n_theta_is_unsupported():
    # n_theta = ceil(16 c R) = 107 is odd: the half-ring symmetry of the kernels needs it even
    with pytest.raises(FBError, match="unsupported"):
        Plan(40, 1 / 3, 20, device=False)


def test_noalloc_scratch_limit_and_host_plan():
    """fb_expand_noalloc checks first that one pass of 16 images fits its fixed 256 MiB array:
    L = 1024 (grid side 2048, 33.7 MB of pass buffers per image) does not, L = 768 (14.3 MB)
    does and then meets the host-only plan."""
    lib = _lib.lib()
    big = Plan(1024, 0.5, 32, device=False)
    assert lib.fb_expand_noalloc(big._h, 1, 1, 1, 0, None) == -7
    assert b"scratch" in lib.fb_error_string(-7)
    ok = Plan(768, 0.5, 32, device=False)
    assert lib.fb_expand_noalloc(ok._h, 1, 1, 1, 0, None) == -5
    assert lib.fb_expand_noalloc(ok._h, 1, -1, 1, 0, None) == -1     # n < 0
    assert lib.fb_expand_noalloc(ok._h, 1, 1, 1, 5, None) == -1      # bad precision
    assert lib.fb_expand_noalloc(None, 1, 1, 1, 0, None) == -1
