"""The rotation-factored M2L (m2l_shape = 3: rotate to the offset's axis,
translate along it, rotate back) against the oracle and against the dense
translation it factors.

The factorization is exact (the CPU test in test_library_cpu.py checks
B T_z A against every dense operator to 1e-12 of its rows), so the two
kernels differ only in rounding order: products agree to 1e-12 relative,
and against the oracle the rotation form meets the bounds of the dense
form (test_gpu_parity.py)."""
import numpy as np
import pytest

import oracle
from paper_1905_01341_amd import bfm
from paper_1905_01341_amd import workload as wl

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def maxrel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.fixture(scope="module")
def c100():
    cl, phi = wl.make("c100")
    s, n, _ = oracle.geometry(cl.xyz, cl.tri)
    rows = wl.subset_rows(cl.nv, 10000, 77)
    ref_l = oracle.offdiag_mvp(cl.xyz, s, n, 1.0, phi, rows=rows)
    ref_m = oracle.offdiag_mvp(cl.xyz, s, n, 0.0, None, 1.0, phi, rows=rows)
    d = oracle.sums(cl.xyz, s, n, phi, rows=rows)
    return cl, phi, s, n, rows, ref_l, ref_m, d


def _solver(cl, **kw):
    sv = bfm.Solver(**kw)
    sv.set_cluster(cl)
    return sv


@pytest.mark.parametrize("orders", [0, 1])
@pytest.mark.parametrize("p", [8, 12, 16, 20])
def test_rotation_m2l_product(c100, p, orders):
    cl, phi, s, n, rows, ref_l, ref_m, _ = c100
    dense = _solver(cl, p=p, m2l_shape=1, m2l_orders=orders)
    rot = _solver(cl, p=p, m2l_shape=3, m2l_orders=orders)
    out = {}
    for name, sv in (("dense", dense), ("rot", rot)):
        out[name] = (sv.matvec(1.0, phi), sv.matvec(0.0, None, 1.0, phi))
    assert rot.tree_stats()["m2l_shape"] == 3
    (dl, dm), (rl, rm) = out["dense"], out["rot"]
    print(f"p={p} orders={orders}: rot vs dense L={rel(rl, dl):.2e} M={rel(rm, dm):.2e}; "
          f"vs oracle L={rel(rl[rows], ref_l):.3e} M={rel(rm[rows], ref_m):.3e} "
          f"max L={maxrel(rl[rows], ref_l):.3e} M={maxrel(rm[rows], ref_m):.3e}")
    assert maxrel(rl, dl) < 1e-12 and maxrel(rm, dm) < 1e-12
    tol_l = {8: 5e-5, 12: 2e-6, 16: 2e-7, 20: 1e-7}[p]
    tol_m = {8: 1e-3, 12: 5e-5, 16: 3e-6, 20: 1e-6}[p]
    e_l, e_m = rel(rl[rows], ref_l), rel(rm[rows], ref_m)
    assert e_l < tol_l and e_m < tol_m, (e_l, e_m)
    assert maxrel(rl[rows], ref_l) < 5 * tol_l and maxrel(rm[rows], ref_m) < 5 * tol_m


def test_rotation_m2l_single_bubble():
    """One sphere at lmax = 2: every far interaction at the minimum separation."""
    cl, phi = wl.make("single")
    s, n, _ = oracle.geometry(cl.xyz, cl.tri)
    x = np.cos(np.arange(cl.nv) * 0.37)
    ref = oracle.offdiag_mvp(cl.xyz, s, n, 1.0, x)
    for p, tol in ((16, 1e-6), (20, 2e-7)):
        dense = _solver(cl, p=p, leaf_target=16, m2l_shape=1).matvec(1.0, x)
        rot = _solver(cl, p=p, leaf_target=16, m2l_shape=3).matvec(1.0, x)
        print(f"p={p}: rot vs dense {maxrel(rot, dense):.2e}, vs oracle {rel(rot, ref):.3e}")
        assert maxrel(rot, dense) < 1e-12 and rel(rot, ref) < tol


def test_rotation_m2l_diagonals(c100):
    """The five-channel pass (p_diag = 20, reduced orders) through the rotation
    kernel: the same M_ii, L_ii and b as the dense pass to rounding, and the
    oracle's to the bounds of test_gpu_parity.py."""
    cl, phi, s, n, rows, _, _, d = c100
    M_ref, L_ref, _ = oracle.diagonals(cl.xyz, s, n, rows=rows, sm=d)
    b_ref = oracle.rhs(phi, d["B"], rows=rows)
    res = {}
    for shape in (1, 3):
        sv = _solver(cl, p=16, m2l_shape=shape, m2l_orders=1)
        res[shape] = sv.diagonals(phi)
        if shape == 3:
            assert sv.tree_stats()["diag_m2l_shape"] == 3
    (M1, L1, b1), (M3, L3, b3) = res[1], res[3]
    print(f"rot vs dense: M={np.abs(M3 - M1).max():.2e} L={maxrel(L3, L1):.2e} b={maxrel(b3, b1):.2e}")
    assert np.abs(M3 - M1).max() < 1e-12 and maxrel(L3, L1) < 1e-9 and maxrel(b3, b1) < 1e-12
    em, el, eb = np.abs(M3[rows] - M_ref).max() / 0.5, rel(L3[rows], L_ref), rel(b3[rows], b_ref)
    print(f"rot vs oracle: M={em:.3e} L={el:.3e} b={eb:.3e}")
    assert em < 1e-6 and el < 1e-6 and eb < 1e-6


def test_rotation_m2l_solve(c100):
    """A refined, preconditioned solve with the rotation kernel in its FP64
    products and diagonal pass satisfies the oracle's system at the rows."""
    cl, phi, s, n, rows, _, _, d = c100
    sv = _solver(cl, p=16, m2l_shape=3, m2l_orders=1, precision=bfm.PREC_BF16X3, p_lo=8,
                 gmres_tol=1e-9, precond=bfm.PRECOND_SH_COARSE, precond_degree=12)
    q, info = sv.solve(phi)
    _, Lii, _ = oracle.diagonals(cl.xyz, s, n, rows=rows, sm=d)
    b = oracle.rhs(phi, d["B"], rows=rows)
    Lq = oracle.offdiag_mvp(cl.xyz, s, n, 1.0, q, rows=rows) + Lii * q[rows]
    print(f"{info['iterations']} it, oracle-system residual {rel(Lq, b):.3e} max {maxrel(Lq, b):.3e}")
    assert info["converged"] and rel(Lq, b) < 1e-6 and maxrel(Lq, b) < 5e-6
