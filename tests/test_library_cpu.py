"""CPU-only checks of the HIP library: it loads, exports every symbol its
headers declare, validates arguments without a GPU, and its host-built
translation operators agree with independent expansions evaluated here.

The expansions in this file are written directly from the Laplace
addition theorem (1/|r - r'| = sum conj(R_n^m(r')) I_n^m(r) over
normalised solid harmonics), not taken from the library.
"""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_1905_01341_amd import bfm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        for m in re.finditer(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(bfm_[a-z_0-9]+)\s*\(", text, re.M):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    lib = bfm.load()
    names = _declared_functions()
    assert len(names) >= 30 and "bfm_mlp_fit" in names and "bfm_mlp_gradient" in names
    for name in names:
        assert hasattr(lib, name), name


def test_default_options_and_errors_without_gpu():
    o = bfm.default_options()
    assert o.abi_version == bfm.ABI_VERSION and o.p == 16 and o.p_diag == 0 and o.gmres_restart == 30
    assert o.p2p_shape == -1 and o.m2l_shape == -1 and o.near_corr == 0
    lib = bfm.load()
    # null arguments are rejected with EINVAL and a message
    assert lib.bfm_create(None, None) == -1
    assert b"null" in lib.bfm_last_error()
    bad = bfm.default_options(p=10)
    h = ctypes.c_void_p()
    assert lib.bfm_create(ctypes.byref(bad), ctypes.byref(h)) == -1
    assert b"multiple of 4" in lib.bfm_last_error()


# --- independent normalised solid harmonics (complex, all orders) -------------

def _nu(n, m):
    m = abs(m)
    return math.sqrt(math.factorial(n - m) * math.factorial(n + m))


def _harm(p, v, irregular):
    """R~ (or I~) for n < p, m = -n..n, via the Legendre form."""
    x, y, z = v
    r = math.sqrt(x * x + y * y + z * z)
    ct = z / r
    st = math.sqrt(max(0.0, 1.0 - ct * ct))
    az = math.atan2(y, x)
    # associated Legendre without Condon-Shortley phase
    P = np.zeros((p, p))
    for m in range(p):
        P[m, m] = math.prod(range(1, 2 * m, 2)) * st ** m if m > 0 else 1.0
        if m + 1 < p:
            P[m + 1, m] = (2 * m + 1) * ct * P[m, m]
        for n in range(m + 2, p):
            P[n, m] = ((2 * n - 1) * ct * P[n - 1, m] - (n + m - 1) * P[n - 2, m]) / (n - m)
    out = {}
    for n in range(p):
        for m in range(0, n + 1):
            e = complex(math.cos(m * az), math.sin(m * az))
            if irregular:
                val = math.factorial(n - m) * P[n, m] * e / (_nu(n, m) * r ** (n + 1))
            else:
                val = _nu(n, m) * r ** n * P[n, m] * e / math.factorial(n + m)
            out[(n, m)] = val
            if m > 0:
                out[(n, -m)] = (-1) ** m * val.conjugate()
    return out


def _pack(coef, p):
    out = np.zeros(p * p)
    for n in range(p):
        out[n * n] = coef[(n, 0)].real
        for m in range(1, n + 1):
            out[n * n + 2 * m - 1] = coef[(n, m)].real
            out[n * n + 2 * m] = coef[(n, m)].imag
    return out


def _unpack(vec, p):
    c = {}
    for n in range(p):
        c[(n, 0)] = complex(vec[n * n], 0.0)
        for m in range(1, n + 1):
            c[(n, m)] = complex(vec[n * n + 2 * m - 1], vec[n * n + 2 * m])
            c[(n, -m)] = (-1) ** m * c[(n, m)].conjugate()
    return c


def _p2m(p, pts, q, c, h):
    acc = {}
    for r, qq in zip(pts, q):
        R = _harm(p, (r - c) / h, False)
        for k, v in R.items():
            acc[k] = acc.get(k, 0.0) + qq * v.conjugate()
    return _pack(acc, p)


def _m2p(p, M, c, h, r):
    I = _harm(p, (r - c) / h, True)
    C = _unpack(M, p)
    return sum(C[k] * I[k] for k in C).real / h


def _p2l(p, pts, q, c, h):
    acc = {}
    for r, qq in zip(pts, q):
        I = _harm(p, (r - c) / h, True)
        for k, v in I.items():
            acc[k] = acc.get(k, 0.0) + qq * v.conjugate()
    return _pack(acc, p)


def _l2p(p, L, c, h, r):
    R = _harm(p, (r - c) / h, False)
    C = _unpack(L, p)
    return sum(C[k] * R[k] for k in C).real / h


def _direct(pts, q, r):
    return sum(qq / np.linalg.norm(r - x) for x, qq in zip(pts, q))


@pytest.mark.parametrize("octant", [0, 3, 5, 7])
def test_m2m_is_exact_reexpansion(octant):
    p, h = 8, 0.7
    rng = np.random.default_rng(octant)
    e = np.array([(octant >> 2) & 1, (octant >> 1) & 1, octant & 1]) - 0.5
    cp = np.array([0.3, -1.0, 2.0])
    cc = cp + e * h
    pts = cc + rng.uniform(-0.5, 0.5, (12, 3)) * h
    q = rng.standard_normal(12)
    T, _ = bfm.debug_operator(p, 0, octant)
    Mc = _p2m(p, pts, q, cc, h)
    Mp = _p2m(p, pts, q, cp, 2 * h)
    np.testing.assert_allclose(T @ Mc, Mp, rtol=1e-12, atol=1e-13 * np.abs(Mp).max())
    # and the parent expansion reproduces the far potential
    tgt = cp + np.array([5.0, -4.0, 6.0])
    assert abs(_m2p(p, Mp, cp, 2 * h, tgt) / _direct(pts, q, tgt) - 1) < 1e-6


@pytest.mark.parametrize("octant", [1, 2, 4, 6])
def test_l2l_is_exact_reexpansion(octant):
    p, h = 8, 0.5
    rng = np.random.default_rng(10 + octant)
    e = np.array([(octant >> 2) & 1, (octant >> 1) & 1, octant & 1]) - 0.5
    cp = np.array([1.0, 2.0, -0.5])
    cc = cp + e * h
    far = cp + np.array([7.0, -6.0, 5.0]) + rng.uniform(-1, 1, (10, 3))
    q = rng.standard_normal(10)
    Lp = _p2l(p, far, q, cp, 2 * h)
    T, _ = bfm.debug_operator(p, 1, octant)
    Lc = T @ Lp
    for r in cc + rng.uniform(-0.5, 0.5, (5, 3)) * h:
        a = _l2p(p, Lp, cp, 2 * h, r)
        b = _l2p(p, Lc, cc, h, r)
        assert abs(a - b) <= 1e-12 * abs(a)


def test_m2l_converges_geometrically():
    """M2L + L2P against the direct sum for a well-separated pair; the error
    falls geometrically with p (cf. the paper's Table 1 trend)."""
    rng = np.random.default_rng(4)
    h = 1.0
    errs = []
    far = next(k for k in range(316) if tuple(bfm.debug_operator(4, 2, k)[1]) == (-3, -3, -3))
    for p in (4, 8, 12):
        for op in (far, 100, 0):
            T, d = bfm.debug_operator(p, 2, op)
            cs = np.zeros(3)
            ct = cs + d * h
            pts = cs + rng.uniform(-0.5, 0.5, (10, 3)) * h
            q = rng.uniform(0.5, 1.0, 10)
            Lt = T @ _p2m(p, pts, q, cs, h)
            e = 0.0
            for r in ct + rng.uniform(-0.5, 0.5, (4, 3)) * h:
                e = max(e, abs(_l2p(p, Lt, ct, h, r) / _direct(pts, q, r) - 1))
            if op == far:
                errs.append(e)
    assert errs[1] < errs[0] / 20 and errs[2] < errs[1] / 20, errs
    assert errs[2] < 1e-6


def test_m2l_offset_enumeration():
    """316 distinct far offsets, numbered nearest first (by |d|^2), so that
    each distance class of the reduced-order M2L is a contiguous range."""
    seen = set()
    d2 = []
    for op in range(316):
        _, d = bfm.debug_operator(4, 2, op)
        assert np.abs(d).max() >= 2 and np.abs(d).max() <= 3
        seen.add(tuple(d))
        d2.append(int(d @ d))
    assert len(seen) == 316
    assert d2 == sorted(d2) and d2[0] == 4 and d2[-1] == 27
    # class boundaries: |d|^2 <= 5 (30 offsets), 6..10 (90), >= 11 (196)
    assert sum(v <= 5 for v in d2) == 30 and sum(6 <= v <= 10 for v in d2) == 90
    with pytest.raises(bfm.BfmError):
        bfm.debug_operator(4, 2, 316)


def _rot_dense(p, A, Tz, B):
    """B T_z A assembled as dense p^2 x p^2 matrices (packed layout)."""
    P = p * p
    Ad, Bd, Td = np.zeros((P, P)), np.zeros((P, P)), np.zeros((P, P))
    for n in range(p):
        sl = slice(n * n, (n + 1) * (n + 1))
        Ad[sl, sl], Bd[sl, sl] = A[n], B[n]
    for m in range(p):
        for part in ((0,) if m == 0 else (0, 1)):
            idx = [j * j + (0 if m == 0 else 2 * m - 1 + part) for j in range(m, p)]
            Td[np.ix_(idx, idx)] = Tz[m]
    return Bd @ Td @ Ad


@pytest.mark.parametrize("p", [4, 8, 16, 20])
def test_m2l_rotation_factorisation(p):
    """T(d) = B T_z(|d|) A for the rotation-factored M2L: rotations block
    diagonal by degree, the translation along the axis coupling equal orders
    only, the product equal to the dense operator (itself checked against
    independent addition-theorem code above) to 1e-12 of every output
    degree's block of rows. (Single rows can be far smaller than their
    degree's block - the order-m rows of a distant operator fall like
    1/sqrt((2m)!) - and a rotation's rounding mixes the block's rows, so a
    row's own relative error can be large while its absolute error stays at
    the block's rounding level.)"""
    ops = range(316) if p <= 16 else range(0, 316, 9)
    worst = 0.0
    for op in ops:
        T, d = bfm.debug_operator(p, 2, op)
        A, Tz, B, d2 = bfm.debug_m2l_rotation(p, op)
        assert tuple(d2) == tuple(d)
        R = _rot_dense(p, A, Tz, B)
        for j in range(p):
            sl = slice(j * j, (j + 1) * (j + 1))
            worst = max(worst, float(np.linalg.norm(R[sl] - T[sl]) / np.linalg.norm(T[sl])))
    assert worst < 1e-12, worst
    # a rotation preserves the degree-n quadratic form with weights 1, 2, 2, ...
    # (the packed parts of orders m > 0 stand for m and -m)
    A, _, B, _ = bfm.debug_m2l_rotation(p, 100)
    for n in (1, p // 2, p - 1):
        w = np.array([1.0] + [2.0] * (2 * n))
        assert np.allclose(A[n].T @ np.diag(w) @ A[n], np.diag(w), atol=1e-12)
