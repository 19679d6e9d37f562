"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Tolerances. The all-pairs GPU product and the geometry agree with the
oracle to round-off. Every comparison is made twice: as a relative 2-norm
over the compared entries (rel) and entry by entry, as the largest error
against the largest reference entry (maxrel), so that a few bad receivers
(one lost or doubled near-field piece) cannot hide in a norm. The
100-bubble products are checked on a fixed seeded subset of 10,000
receivers against the oracle's exact sums over all 256,200 sources. Fast multipole products carry the truncation error of
expansions of degree < p with one-box separation (geometric in p, cf. the
paper's Table 1): single layer (L) within 1e-6 from p = 16, double layer
(M, dipoles, one order slower) within 1e-6 from p = 20, which is why the
once-per-solve pass for the diagonals and b runs at p_diag = 20.
"""
import numpy as np
import pytest

import oracle
from paper_1905_01341_amd import bfm
from paper_1905_01341_amd import workload as wl

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def maxrel(a, b):
    """Largest entry-wise error against the largest reference entry."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.fixture(scope="module")
def single():
    cl, phi = wl.make("single")
    s, n, _ = oracle.geometry(cl.xyz, cl.tri)
    return cl, phi, s, n


@pytest.fixture(scope="module")
def c100():
    cl, phi = wl.make("c100")
    s, n, _ = oracle.geometry(cl.xyz, cl.tri)
    rows = wl.subset_rows(cl.nv, 10000, 77)
    return cl, phi, s, n, rows


@pytest.fixture(scope="module")
def c100_ref(c100):
    """The oracle's single- and double-layer products with phi and its
    diagonal/right-hand-side sums at the 10,000 sampled receivers."""
    cl, phi, s, n, rows = c100
    ref_l = oracle.offdiag_mvp(cl.xyz, s, n, 1.0, phi, rows=rows)
    ref_m = oracle.offdiag_mvp(cl.xyz, s, n, 0.0, None, 1.0, phi, rows=rows)
    d = oracle.sums(cl.xyz, s, n, phi, rows=rows)
    return ref_l, ref_m, d


def _solver(cl, **kw):
    sv = bfm.Solver(**kw)
    sv.set_cluster(cl)
    return sv


def test_geometry_matches_oracle(single, c100):
    for cl, s_ref, n_ref in ((single[0], single[2], single[3]), (c100[0], c100[2], c100[3])):
        sv = _solver(cl)
        s, n = sv.geometry()
        np.testing.assert_allclose(s, s_ref, rtol=1e-13)
        np.testing.assert_allclose(n, n_ref, rtol=0, atol=1e-13)


def test_direct_product_matches_oracle(single):
    cl, phi, s, n = single
    sv = _solver(cl)
    x = np.cos(np.arange(cl.nv) * 0.37)
    yl = sv.matvec(1.0, x, direct=True)
    ym = sv.matvec(0.0, None, 1.0, phi, direct=True)
    np.testing.assert_allclose(yl, oracle.offdiag_mvp(cl.xyz, s, n, 1.0, x), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(ym, oracle.offdiag_mvp(cl.xyz, s, n, 0.0, None, 1.0, phi),
                               rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("p", [8, 12, 16, 20])
def test_fmm_product_single_bubble(single, p):
    """One sphere, lmax = 2: every far interaction is at the minimum
    separation, the worst case of the expansion error."""
    cl, phi, s, n = single
    sv = _solver(cl, p=p, leaf_target=16)
    x = np.cos(np.arange(cl.nv) * 0.37)
    ref_l = oracle.offdiag_mvp(cl.xyz, s, n, 1.0, x)
    ref_m = oracle.offdiag_mvp(cl.xyz, s, n, 0.0, None, 1.0, phi)
    yl, ym = sv.matvec(1.0, x), sv.matvec(0.0, None, 1.0, phi)
    e_l, e_m = rel(yl, ref_l), rel(ym, ref_m)
    x_l, x_m = maxrel(yl, ref_l), maxrel(ym, ref_m)
    print(f"p={p} L={e_l:.3e} M={e_m:.3e} max L={x_l:.3e} M={x_m:.3e}")
    tol = {8: 2e-4, 12: 1e-5, 16: 1e-6, 20: 2e-7}[p]
    assert e_l < tol and e_m < 2 * tol, (p, e_l, e_m)
    assert x_l < 5 * tol and x_m < 10 * tol, (p, x_l, x_m)


@pytest.mark.parametrize("p", [8, 12, 16, 20])
def test_fmm_product_cluster_sampled(c100, c100_ref, p):
    """256,200 sources; the oracle sums 10,000 sampled receivers exactly."""
    cl, phi, s, n, rows = c100
    ref_l, ref_m, _ = c100_ref
    sv = _solver(cl, p=p)
    yl = sv.matvec(1.0, phi)
    ym = sv.matvec(0.0, None, 1.0, phi)
    e_l, e_m = rel(yl[rows], ref_l), rel(ym[rows], ref_m)
    x_l, x_m = maxrel(yl[rows], ref_l), maxrel(ym[rows], ref_m)
    print(f"p={p} L={e_l:.3e} M={e_m:.3e} max L={x_l:.3e} M={x_m:.3e}")
    tol_l = {8: 5e-5, 12: 2e-6, 16: 2e-7, 20: 1e-7}[p]
    tol_m = {8: 1e-3, 12: 5e-5, 16: 3e-6, 20: 1e-6}[p]
    assert e_l < tol_l and e_m < tol_m, (p, e_l, e_m)
    assert x_l < 5 * tol_l and x_m < 5 * tol_m, (p, x_l, x_m)


@pytest.mark.parametrize("p", [12, 16, 20])
def test_reduced_order_m2l_matches_full_order_bounds(c100, c100_ref, p):
    """M2L of distant offsets at reduced orders (m2l_orders = 1: |d|^2 <= 5 at
    p, 6..10 at 4 ceil(p/5), >= 11 at 4 ceil(3p/20)) keeps the full-order
    product's accuracy: the same 2-norm and entry-wise bounds as
    test_fmm_product_cluster_sampled."""
    cl, phi, s, n, rows = c100
    ref_l, ref_m, _ = c100_ref
    sv = _solver(cl, p=p, m2l_orders=1)
    yl = sv.matvec(1.0, phi)
    ym = sv.matvec(0.0, None, 1.0, phi)
    e_l, e_m = rel(yl[rows], ref_l), rel(ym[rows], ref_m)
    x_l, x_m = maxrel(yl[rows], ref_l), maxrel(ym[rows], ref_m)
    print(f"p={p} reduced orders: L={e_l:.3e} M={e_m:.3e} max L={x_l:.3e} M={x_m:.3e}")
    tol_l = {12: 2e-6, 16: 2e-7, 20: 1e-7}[p]
    tol_m = {12: 5e-5, 16: 3e-6, 20: 1e-6}[p]
    assert e_l < tol_l and e_m < tol_m, (p, e_l, e_m)
    assert x_l < 5 * tol_l and x_m < 5 * tol_m, (p, x_l, x_m)


def test_reduced_order_diagonals_and_rhs(c100, c100_ref):
    """The five-channel pass (p_diag = 20) with reduced-order distant
    translations against the full-order pass, both against the oracle:
    M_ii, L_ii and b within the same 2-norm bounds, and entry-wise within
    twice the full-order pass's error (L_ii, a small difference of sums of
    coordinates relative to the cube centre, is the channel most sensitive
    to the expansion order)."""
    cl, phi, s, n, rows = c100
    d = c100_ref[2]
    M_ref, L_ref, _ = oracle.diagonals(cl.xyz, s, n, rows=rows, sm=d)
    b_ref = oracle.rhs(phi, d["B"], rows=rows)
    errs = {}
    for orders in (0, 1):
        sv = _solver(cl, p=16, m2l_orders=orders)
        Mii, Lii, b = sv.diagonals(phi)
        errs[orders] = (np.abs(Mii[rows] - M_ref).max() / 0.5, rel(Lii[rows], L_ref), rel(b[rows], b_ref),
                        maxrel(Lii[rows], L_ref), maxrel(b[rows], b_ref))
        print("orders=%d: M=%.3e L=%.3e b=%.3e max L=%.3e b=%.3e" % ((orders,) + errs[orders]))
    em, el, eb, xl, xb = errs[1]
    assert em < 1e-6 and el < 1e-6 and eb < 1e-6, errs[1]
    assert em <= 2 * errs[0][0] + 1e-12 and xl <= 2 * errs[0][3] and xb <= 2 * errs[0][4] + 1e-12, errs


@pytest.mark.parametrize("lmax", [3, 4])
def test_fmm_product_coarse_and_fine_leaves(c100, c100_ref, lmax):
    """Fixed octree depths on the 100-bubble cluster: at lmax = 3 every
    leaf's near-field source list runs to thousands of points and is split
    into pieces whose sums are added atomically; at lmax = 4 the lists are
    shorter. Both must give the same product to the expansion accuracy."""
    cl, phi, s, n, rows = c100
    ref_l, ref_m, _ = c100_ref
    sv = _solver(cl, p=16, lmax=lmax)
    st = sv.tree_stats()
    assert st["lmax"] == lmax
    yl = sv.matvec(1.0, phi)
    ym = sv.matvec(0.0, None, 1.0, phi)
    e_l, e_m = rel(yl[rows], ref_l), rel(ym[rows], ref_m)
    x_l, x_m = maxrel(yl[rows], ref_l), maxrel(ym[rows], ref_m)
    print(f"lmax={lmax} near pairs={st['near_pairs']} L={e_l:.3e} M={e_m:.3e} max L={x_l:.3e} M={x_m:.3e}")
    assert e_l < 2e-7 and e_m < 3e-6, (lmax, e_l, e_m)
    assert x_l < 1e-6 and x_m < 1.5e-5, (lmax, x_l, x_m)


def test_fmm_product_tiny_leaves(single):
    """One sphere at lmax = 5: leaves of a few points, near-field source
    lists short enough to stay in one piece (stores instead of atomics).
    Nearly every far interaction of this tree is at the minimum separation,
    so the truncation error at p = 16 is larger than at lmax = 2 (measured
    1.1e-6 for L and 6.8e-6 for M); a lost or doubled near-field piece
    would show as an error of order one."""
    cl, phi, s, n = single
    sv = _solver(cl, p=16, lmax=5)
    x = np.cos(np.arange(cl.nv) * 0.37)
    ref_l, ref_m = oracle.offdiag_mvp(cl.xyz, s, n, 1.0, x), oracle.offdiag_mvp(cl.xyz, s, n, 0.0, None, 1.0, phi)
    yl, ym = sv.matvec(1.0, x), sv.matvec(0.0, None, 1.0, phi)
    e_l, e_m, x_l, x_m = rel(yl, ref_l), rel(ym, ref_m), maxrel(yl, ref_l), maxrel(ym, ref_m)
    print(f"L={e_l:.3e} M={e_m:.3e} max L={x_l:.3e} M={x_m:.3e}")
    assert e_l < 3e-6 and e_m < 2e-5, (e_l, e_m)
    assert x_l < 1.5e-5 and x_m < 1e-4, (x_l, x_m)


def test_fmm_product_deep_octree(single):
    """One sphere at lmax = 11, deeper than the levels the first key sort
    orders (10): the points are sorted by all 45 key bits and every leaf
    holds at most a few points. The product must still match the oracle to
    the expansion accuracy (limits as for the tiny leaves above)."""
    cl, phi, s, n = single
    sv = _solver(cl, p=16, lmax=11)
    assert sv.tree_stats()["lmax"] == 11
    x = np.cos(np.arange(cl.nv) * 0.37)
    ref_l, ref_m = oracle.offdiag_mvp(cl.xyz, s, n, 1.0, x), oracle.offdiag_mvp(cl.xyz, s, n, 0.0, None, 1.0, phi)
    yl, ym = sv.matvec(1.0, x), sv.matvec(0.0, None, 1.0, phi)
    e_l, e_m, x_l, x_m = rel(yl, ref_l), rel(ym, ref_m), maxrel(yl, ref_l), maxrel(ym, ref_m)
    print(f"L={e_l:.3e} M={e_m:.3e} max L={x_l:.3e} M={x_m:.3e}")
    assert e_l < 3e-6 and e_m < 2e-5, (e_l, e_m)
    assert x_l < 1.5e-5 and x_m < 1e-4, (x_l, x_m)


def test_diagonals_and_rhs(single, c100, c100_ref):
    """M_ii = -1/2 - sum M_ij is a small difference of O(1/2) terms, so its
    error is judged against 1/2 (the size of the sum it comes from)."""
    cl, phi, s, n = single
    sv = _solver(cl, p=16, leaf_target=16)  # p_diag = 20
    Mii, Lii, b = sv.diagonals(phi)
    d = oracle.sums(cl.xyz, s, n, phi)
    M_ref, L_ref, _ = oracle.diagonals(cl.xyz, s, n, sm=d)
    b_ref = oracle.rhs(phi, d["B"])
    em, el, eb = np.abs(Mii - M_ref).max() / 0.5, rel(Lii, L_ref), rel(b, b_ref)
    xl, xb = maxrel(Lii, L_ref), maxrel(b, b_ref)
    print(f"single: M={em:.3e} L={el:.3e} b={eb:.3e} max L={xl:.3e} b={xb:.3e}")
    assert em < 1e-6 and el < 1e-6 and eb < 1e-6, (em, el, eb)
    assert xl < 5e-6 and xb < 5e-6, (xl, xb)
    cl, phi, s, n, rows = c100
    d = c100_ref[2]
    sv = _solver(cl, p=16)
    Mii, Lii, b = sv.diagonals(phi)
    M_ref, L_ref, _ = oracle.diagonals(cl.xyz, s, n, rows=rows, sm=d)
    b_ref = oracle.rhs(phi, d["B"], rows=rows)
    em, el, eb = np.abs(Mii[rows] - M_ref).max() / 0.5, rel(Lii[rows], L_ref), rel(b[rows], b_ref)
    xl, xb = maxrel(Lii[rows], L_ref), maxrel(b[rows], b_ref)
    print(f"c100: M={em:.3e} L={el:.3e} b={eb:.3e} max L={xl:.3e} b={xb:.3e}")
    assert em < 1e-6 and el < 1e-6 and eb < 1e-6, (em, el, eb)
    assert xl < 5e-6 and xb < 5e-6, (xl, xb)


def test_solve_single_bubble_matches_oracle(single):
    cl, phi, s, n = single
    q_ref, _ = oracle.solve(cl.xyz, cl.tri, phi, method="lu")
    sv = _solver(cl, p=16, leaf_target=16, gmres_tol=1e-12)
    q, info = sv.solve(phi)
    assert info["converged"]
    assert rel(q, q_ref) < 1e-6, (rel(q, q_ref), info)
    assert maxrel(q, q_ref) < 5e-6, maxrel(q, q_ref)


def test_solve_cluster_residual_against_oracle_rows(c100, c100_ref):
    """The GPU solution satisfies the oracle's system at sampled rows."""
    cl, phi, s, n, rows = c100
    sv = _solver(cl, p=16, gmres_tol=1e-10)
    q, info = sv.solve(phi)
    assert info["converged"], info
    d = c100_ref[2]
    _, Lii, _ = oracle.diagonals(cl.xyz, s, n, rows=rows, sm=d)
    b = oracle.rhs(phi, d["B"], rows=rows)
    Lq = oracle.offdiag_mvp(cl.xyz, s, n, 1.0, q, rows=rows) + Lii * q[rows]
    print(f"residual of the GPU solution in the oracle system: {rel(Lq, b):.3e} "
          f"max {maxrel(Lq, b):.3e} ({info})")
    assert rel(Lq, b) < 1e-6 and maxrel(Lq, b) < 5e-6, (rel(Lq, b), maxrel(Lq, b))


def test_warm_start_and_tetrahedron_edge_cases():
    # smallest closed surface: a tetrahedron (4 vertices, 4 triangles)
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float)
    f = np.array([[0, 1, 2], [0, 3, 1], [0, 2, 3], [1, 3, 2]], np.int32)
    cr = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])
    assert np.all(np.einsum("ij,ij->i", cr, v[f].mean(1)) > 0)
    phi = np.array([1.0, 0.5, -0.25, 2.0])
    q_ref, _ = oracle.solve(v, f, phi, method="lu")
    dirs = v / np.linalg.norm(v, axis=1, keepdims=True)
    sv = _solver(wl.Cluster(v, f, np.array([0, 4]), np.array([0, 4]), np.zeros((1, 3)), np.ones(1), dirs),
                 p=16, gmres_tol=1e-13)
    q, info = sv.solve(phi)
    assert rel(q, q_ref) < 1e-6 and maxrel(q, q_ref) < 5e-6, (rel(q, q_ref), maxrel(q, q_ref))
    # warm start from the answer converges immediately
    q2, info2 = sv.solve(phi, q0=q)
    assert info2["iterations"] <= 1 and rel(q2, q) < 1e-12


def test_degenerate_mesh_is_rejected():
    cl, phi = wl.make("single")
    tri = cl.tri.copy()
    tri[5, 2] = tri[5, 1]
    sv = bfm.Solver()
    sv.set_mesh(cl.xyz, tri)
    with pytest.raises(bfm.BfmError) as e:
        sv.solve(phi)
    assert e.value.code == -5


def test_sh_preconditioned_solve_single_bubble(single):
    """Right preconditioning leaves the solution unchanged and cuts the
    iteration count (the single layer is nearly diagonal in harmonics)."""
    cl, phi, s, n = single
    q_ref, _ = oracle.solve(cl.xyz, cl.tri, phi, method="lu")
    plain = _solver(cl, p=16, leaf_target=16, gmres_tol=1e-12)
    q0, i0 = plain.solve(phi)
    pre = _solver(cl, p=16, leaf_target=16, gmres_tol=1e-12, precond=bfm.PRECOND_SH, precond_degree=12)
    q1, i1 = pre.solve(phi)
    print(f"plain {i0['iterations']} it, preconditioned {i1['iterations']} it")
    assert i1["converged"] and rel(q1, q_ref) < 1e-6, (rel(q1, q_ref), i1)
    assert maxrel(q1, q_ref) < 5e-6, maxrel(q1, q_ref)
    assert i1["iterations"] < i0["iterations"] / 2


def test_sh_preconditioned_solve_cluster(c100, c100_ref):
    cl, phi, s, n, rows = c100
    sv = _solver(cl, p=16, gmres_tol=1e-10, precond=bfm.PRECOND_SH, precond_degree=12)
    q, info = sv.solve(phi)
    assert info["converged"], info
    d = c100_ref[2]
    _, Lii, _ = oracle.diagonals(cl.xyz, s, n, rows=rows, sm=d)
    b = oracle.rhs(phi, d["B"], rows=rows)
    Lq = oracle.offdiag_mvp(cl.xyz, s, n, 1.0, q, rows=rows) + Lii * q[rows]
    print(f"preconditioned: {info['iterations']} it, oracle-system residual {rel(Lq, b):.3e} "
          f"max {maxrel(Lq, b):.3e}")
    assert rel(Lq, b) < 1e-6 and maxrel(Lq, b) < 5e-6 and info["iterations"] < 60


def test_two_level_preconditioned_solve_cluster(c100, c100_ref):
    """The coarse correction (one unknown per bubble) leaves the solution
    unchanged and needs fewer iterations than the block step alone."""
    cl, phi, s, n, rows = c100
    sh = _solver(cl, p=16, gmres_tol=1e-10, precond=bfm.PRECOND_SH, precond_degree=12)
    q1, i1 = sh.solve(phi)
    two = _solver(cl, p=16, gmres_tol=1e-10, precond=bfm.PRECOND_SH_COARSE, precond_degree=12)
    q2, i2 = two.solve(phi)
    assert i2["converged"], i2
    d = c100_ref[2]
    _, Lii, _ = oracle.diagonals(cl.xyz, s, n, rows=rows, sm=d)
    b = oracle.rhs(phi, d["B"], rows=rows)
    Lq = oracle.offdiag_mvp(cl.xyz, s, n, 1.0, q2, rows=rows) + Lii * q2[rows]
    print(f"block {i1['iterations']} it, two-level {i2['iterations']} it, "
          f"oracle-system residual {rel(Lq, b):.3e} max {maxrel(Lq, b):.3e}")
    assert rel(Lq, b) < 1e-6 and maxrel(Lq, b) < 5e-6
    assert rel(q2, q1) < 1e-8
    assert i2["iterations"] < i1["iterations"]
    # the second solve on the same mesh reuses nothing stale: positions moved
    xyz = cl.xyz * 1.01
    two.set_positions(xyz)
    sh.set_positions(xyz)
    q3, i3 = two.solve(phi)
    q4, _ = sh.solve(phi)
    assert i3["converged"] and rel(q3, q4) < 1e-8


def test_two_level_solve_after_a_failed_solve(c100):
    """The coarse space is built on a second stream beside the diagonal pass.
    A solve that stops at gmres_maxit (an error) leaves that build without a
    waiter; moving the vertices and solving again must still be exact."""
    cl, phi, s, n, rows = c100
    two = _solver(cl, p=16, gmres_tol=1e-10, gmres_maxit=1, precond=bfm.PRECOND_SH_COARSE,
                  precond_degree=12)
    with pytest.raises(bfm.BfmError):
        two.solve(phi)
    xyz = cl.xyz * 0.99
    two.set_positions(xyz)
    two.set_options(gmres_maxit=500)
    q1, i1 = two.solve(phi)
    fresh = _solver(cl, p=16, gmres_tol=1e-10, precond=bfm.PRECOND_SH_COARSE, precond_degree=12)
    fresh.set_positions(xyz)
    q2, i2 = fresh.solve(phi)
    assert i1["converged"] and i2["converged"]
    assert i1["iterations"] == i2["iterations"] and rel(q1, q2) < 1e-10, (i1, i2, rel(q1, q2))
    # later builds on new positions
    for scale in (1.02, 0.97):
        xyz = cl.xyz * scale
        two.set_positions(xyz)
        fresh.set_positions(xyz)
        q1, i1 = two.solve(phi)
        q2, i2 = fresh.solve(phi)
        assert i1["iterations"] == i2["iterations"] and rel(q1, q2) < 1e-10, (scale, i1, i2, rel(q1, q2))


def test_sphere_template_validation():
    cl, phi = wl.make("single")
    sv = bfm.Solver()
    sv.set_mesh(cl.xyz, cl.tri)
    with pytest.raises(bfm.BfmError):
        sv.set_sphere_template(cl.dirs[:100])  # wrong vertex count
    with pytest.raises(bfm.BfmError):
        sv.set_sphere_template(cl.dirs * 2.0)  # not unit vectors
    sv.set_options(precond=bfm.PRECOND_SH)
    with pytest.raises(bfm.BfmError):
        sv.solve(phi)  # no template set
