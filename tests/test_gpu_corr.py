"""Near-field correction matrices on the GPU (bfm_options.near_corr, Section
3.9) against the oracle (oracle/corrections.py).

The corrections are exact sparse sums, so their part of every product, of the
singular diagonals and of b is compared at FP64 round-off: the difference of
a product with and without them (same octree, same fast multipole sums) is
the correction product alone. Meshes: one regular icosphere (642 vertices,
many equidistant vertices, so the collapse vertex's tie rule is exercised)
and the 100-bubble cluster (sampled rows). Bounds: 1e-12 of the largest
entry for the sparse parts; the corrected solve against the oracle's
corrected direct solve at the fast multipole product's accuracy (2-norm
1e-6, largest entry 5e-6, the nodal solve's bounds).
"""
import numpy as np
import pytest

import oracle
from oracle import corrections as oc
from paper_1905_01341_amd import bfm
from paper_1905_01341_amd import workload as wl

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def maxrel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _vec(nv, k):
    return np.cos(np.arange(nv) * (0.37 + 0.11 * k)) + 0.3 * np.sin(np.arange(nv) * 1.7)


def _rows(cl, name):
    return np.arange(cl.nv) if name == "single" else wl.subset_rows(cl.nv, 300, 5)


@pytest.mark.parametrize("name", ["single", "c100"])
@pytest.mark.parametrize("direct", [False, True])
def test_product_corrections(name, direct):
    """(f L + g M) with minus without corrections = f CL x + g CM y."""
    if name == "c100" and direct:
        pytest.skip("all-pairs product at 256k points: covered by the fast multipole case")
    cl, phi = wl.make(name)
    rows = _rows(cl, name)
    s, n, _ = oracle.geometry(cl.xyz, cl.tri)
    corr = oc.corrections(cl.xyz, cl.tri, s, n, rows=rows)
    x, y = _vec(cl.nv, 0), _vec(cl.nv, 1)
    sv = bfm.Solver(p=16)
    sv.set_cluster(cl)
    for f, g in ((1.0, 0.0), (0.0, 1.0), (0.7, -1.3)):
        xx, yy = (x if f else None), (y if g else None)
        sv.set_options(near_corr=0)
        a = sv.matvec(f, xx, g, yy, direct=direct)
        sv.set_options(near_corr=1)
        b = sv.matvec(f, xx, g, yy, direct=direct)
        ref = oc.apply(corr, f, x, g, y)
        e = float(np.max(np.abs((b - a)[rows] - ref)) / np.max(np.abs(a)))
        print(f"{name} direct={direct} f={f} g={g}: correction error {e:.2e} (|corr| {np.max(np.abs(ref)):.2e})")
        assert e < 1e-12, (f, g, e)
    sv.close()


@pytest.mark.parametrize("name", ["single", "c100"])
def test_diagonal_corrections(name):
    """Corrected M_ii, L_ii and b minus the nodal ones against the oracle's
    row identities applied to its corrections."""
    cl, phi = wl.make(name)
    rows = _rows(cl, name)
    s, n, _ = oracle.geometry(cl.xyz, cl.tri)
    corr = oc.corrections(cl.xyz, cl.tri, s, n, rows=rows)
    z = np.zeros(len(rows))
    dM, dL, db = oc.corrected_diagonals(cl.xyz, n, phi, corr, z, z, z)
    sv = bfm.Solver(p=16)
    sv.set_cluster(cl)
    M0, L0, b0 = sv.diagonals(phi)
    sv.set_options(near_corr=1)
    M1, L1, b1 = sv.diagonals(phi)
    sv.close()
    for got, want, base, tag in ((M1 - M0, dM, M0, "M"), (L1 - L0, dL, L0, "L"), (b1 - b0, db, b0, "b")):
        e = float(np.max(np.abs(got[rows] - want)) / np.max(np.abs(base)))
        print(f"{name} {tag}_ii correction error {e:.2e} (largest correction {np.max(np.abs(want)):.2e})")
        assert e < 1e-12, (tag, e)


def test_corrected_solve_single():
    """The corrected system solved on the GPU against the oracle's corrected
    solve (direct sums), fast multipole and graph-replayed."""
    cl, phi = wl.make("single")
    q_ref, info = oc.solve(cl.xyz, cl.tri, phi, tol=1e-12)
    q_nodal, _ = oracle.solve(cl.xyz, cl.tri, phi, tol=1e-12)
    for graph in (0, 1):
        sv = bfm.Solver(p=16, near_corr=1, gmres_tol=1e-12, use_graph=graph)
        sv.set_cluster(cl)
        q, inf = sv.solve(phi)
        sv.close()
        e, x = rel(q, q_ref), maxrel(q, q_ref)
        print(f"graph={graph}: corrected solve error {e:.2e} (largest {x:.2e}, {inf['iterations']} "
              f"iterations); corrected vs nodal {rel(q_ref, q_nodal):.2e}")
        assert e < 1e-6 and x < 5e-6, (e, x)
        assert rel(q, q_nodal) > 100 * e  # the corrections change the answer


def test_corrected_mixed_precision_solve():
    """FP32 refinement with the corrections reaches the FP64 corrected solve."""
    cl, phi = wl.make("c100")
    out = {}
    for prec in (bfm.PREC_FP64, bfm.PREC_FP32):
        sv = bfm.Solver(p=16, near_corr=1, gmres_tol=1e-10, precision=prec, precond=bfm.PRECOND_SH_COARSE)
        sv.set_cluster(cl)
        out[prec], inf = sv.solve(phi)
        sv.close()
        print(prec, inf["iterations"], inf["rel_residual"])
        assert inf["converged"]
    assert maxrel(out[bfm.PREC_FP32], out[bfm.PREC_FP64]) < 1e-8


def test_corrections_follow_the_mesh():
    """New positions rebuild the values, a new mesh the pattern, and turning
    the option off removes them."""
    cl, phi = wl.make("single")
    x = _vec(cl.nv, 2)
    sv = bfm.Solver(p=16, near_corr=1)
    sv.set_cluster(cl)
    sv.matvec(1.0, x, direct=True)
    moved = cl.xyz * np.array([1.3, 0.9, 1.1]) + 0.2
    sv.set_positions(moved)
    got = sv.matvec(1.0, x, 1.0, x, direct=True)
    s, n, _ = oracle.geometry(moved, cl.tri)
    corr = oc.corrections(moved, cl.tri, s, n)
    ref = oracle.offdiag_mvp(moved, s, n, 1.0, x, 1.0, x) + oc.apply(corr, 1.0, x, 1.0, x)
    assert maxrel(got, ref) < 1e-12
    # a different mesh: two bubbles of a smaller icosphere
    xyz, tri = wl.icosphere(2)
    xyz2 = np.concatenate([xyz, xyz + np.array([3.0, 0.0, 0.0])])
    tri2 = np.concatenate([tri, tri + len(xyz)]).astype(np.int32)
    sv.set_mesh(xyz2, tri2)
    x2 = _vec(len(xyz2), 3)
    got = sv.matvec(0.0, None, 1.0, x2, direct=True)
    s, n, _ = oracle.geometry(xyz2, tri2)
    corr = oc.corrections(xyz2, tri2, s, n)
    ref = oracle.offdiag_mvp(xyz2, s, n, 0.0, None, 1.0, x2) + oc.apply(corr, 0.0, None, 1.0, x2)
    assert maxrel(got, ref) < 1e-12
    sv.set_options(near_corr=0)
    got = sv.matvec(0.0, None, 1.0, x2, direct=True)
    assert maxrel(got, oracle.offdiag_mvp(xyz2, s, n, 0.0, None, 1.0, x2)) < 1e-12
    with pytest.raises(bfm.BfmError):
        sv.set_options(near_corr=2)
    sv.close()


def _bipyramid(n):
    """Closed bipyramid: apexes (0, 0, +-1) over n equator points; each apex
    has n neighbours, so its correction row has n + 1 columns."""
    ang = 2.0 * np.pi * np.arange(n) / n
    xyz = np.concatenate([[[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]],
                          np.stack([np.cos(ang), np.sin(ang), 0.05 * np.sin(3 * ang)], axis=1)])
    tri = []
    for k in range(n):
        a, b = 2 + k, 2 + (k + 1) % n
        tri += [(0, a, b), (1, b, a)]
    return xyz, np.array(tri, dtype=np.int32)


@pytest.mark.parametrize("n", [24, 48])
def test_wide_rows(n):
    """Rows wider than the LDS accumulators hold (48 equator points: 49
    columns at the apexes) take the in-place path; both match the oracle."""
    xyz, tri = _bipyramid(n)
    nv = len(xyz)
    s, nrm, _ = oracle.geometry(xyz, tri)
    corr = oc.corrections(xyz, tri, s, nrm)
    assert max(len(c) for c, _, _ in corr.values()) == n + 1
    x, y = _vec(nv, 4), _vec(nv, 5)
    phi = np.cos(np.arange(nv) * 0.3)
    sv = bfm.Solver(p=16, leaf_target=8)
    sv.set_mesh(xyz, tri)
    a = sv.matvec(0.7, x, -1.3, y, direct=True)
    M0, L0, b0 = sv.diagonals(phi)
    sv.set_options(near_corr=1)
    b = sv.matvec(0.7, x, -1.3, y, direct=True)
    M1, L1, b1 = sv.diagonals(phi)
    sv.close()
    ref = oc.apply(corr, 0.7, x, -1.3, y)
    e = float(np.max(np.abs((b - a) - ref)) / np.max(np.abs(a)))
    z = np.zeros(nv)
    dM, dL, db = oc.corrected_diagonals(xyz, nrm, phi, corr, z, z, z)
    ed = max(float(np.max(np.abs(g - w)) / np.max(np.abs(base)))
             for g, w, base in ((M1 - M0, dM, M0), (L1 - L0, dL, L0), (b1 - b0, db, b0)))
    print(f"bipyramid n={n}: product correction error {e:.2e}, diagonals {ed:.2e}")
    assert e < 1e-12 and ed < 1e-12

