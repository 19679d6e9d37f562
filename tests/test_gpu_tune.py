"""GPU checks of the graph-captured GMRES product and of the autotuner.

The graph path replays one captured product per octree; GMRES runs its own
eager kernels and a host synchronisation between replays, and ends on an
eager true-residual product, so a wrong replay shows up as a different
iteration count or solution. Each solve after moving the vertices captures
a new graph (new octree)."""
import numpy as np
import pytest

from paper_1905_01341_amd import bfm
from paper_1905_01341_amd import workload as wl

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def cluster():
    cl = wl.cluster(60, 3, 35.0, 0.5, 1.0, 0.5, seed=9, perturb=0.05)
    return cl, wl.smooth_phi(cl, 10)


@pytest.mark.parametrize("precond", [bfm.PRECOND_NONE, bfm.PRECOND_SH_COARSE])
def test_graph_solves_match_eager(cluster, precond):
    cl, phi = cluster
    kw = dict(p=16, gmres_tol=1e-11, precond=precond)
    eager = bfm.Solver(**kw)
    eager.set_cluster(cl)
    graph = bfm.Solver(use_graph=1, **kw)
    graph.set_cluster(cl)
    rng = np.random.default_rng(precond)
    for k in range(3):
        xyz = cl.xyz * (1.0 + 0.001 * k) + 0.01 * k * rng.standard_normal(3)
        eager.set_positions(xyz)
        graph.set_positions(xyz)
        qe, ie = eager.solve(phi)
        qg, ig = graph.solve(phi)
        print(f"solve {k}: eager {ie['iterations']} it, graph {ig['iterations']} it, diff {rel(qg, qe):.2e}")
        assert ig["converged"] and abs(ig["iterations"] - ie["iterations"]) <= 1
        assert rel(qg, qe) < 1e-9
        # warm start from the answer on the same graph
        qw, iw = graph.solve(phi, q0=qg)
        assert iw["iterations"] <= 1 and rel(qw, qg) < 1e-10


def test_autotune_choices_and_solution(cluster):
    cl, phi = cluster
    sv = bfm.Solver(gmres_tol=1e-10, precond=bfm.PRECOND_SH_COARSE)
    sv.set_cluster(cl)
    lmax0 = sv.tree_stats()["lmax"]
    r = sv.autotune(1e-7)
    print(r)
    assert r["p"] in (12, 16, 20) and r["p_err"] <= 1e-7
    assert abs(r["lmax"] - lmax0) <= 2 and r["m2l_shape"] in (0, 1, 2, 3)
    assert r["candidates"] >= 8 and r["mvp_ms"] > 0
    assert sv.tree_stats()["lmax"] == r["lmax"]
    # the diagonal pass's order: within 10 x the product tolerance of order 20
    assert r["p_diag"] in (12, 16, 20) and r["p_diag"] >= r["p"] and r["diag_err"] <= 1e-6
    assert sv.opt.p_diag == r["p_diag"]
    q, info = sv.solve(phi)
    ref = bfm.Solver(p=20, gmres_tol=1e-10, precond=bfm.PRECOND_SH_COARSE)
    ref.set_cluster(cl)
    q20, _ = ref.solve(phi)
    assert info["converged"] and rel(q, q20) < 1e-6


def test_autotuned_diagonal_order_against_the_oracle(cluster):
    """The autotuner's p_diag (here chosen among 12, 16, 20) gives diagonals
    within the oracle bounds of the fixed p_diag = 20 pass (M_ii within 1e-6
    of 1/2, L_ii and b within 1e-6 relative)."""
    import oracle
    cl, phi = cluster
    sv = bfm.Solver(gmres_tol=1e-10, precond=bfm.PRECOND_SH_COARSE)
    sv.set_cluster(cl)
    r = sv.autotune(1e-7)
    Mii, Lii, b = sv.diagonals(phi)
    s, n, _ = oracle.geometry(cl.xyz, cl.tri)
    rows = np.arange(0, cl.nv, 7)
    d = oracle.sums(cl.xyz, s, n, phi, rows=rows)
    M_ref, L_ref, _ = oracle.diagonals(cl.xyz, s, n, rows=rows, sm=d)
    b_ref = oracle.rhs(phi, d["B"], rows=rows)
    em, el, eb = np.abs(Mii[rows] - M_ref).max() / 0.5, rel(Lii[rows], L_ref), rel(b[rows], b_ref)
    print(f"p_diag {r['p_diag']} (diag_err {r['diag_err']:.2e}): M={em:.2e} L={el:.2e} b={eb:.2e}")
    assert em < 1e-6 and el < 1e-6 and eb < 1e-6


@pytest.mark.parametrize("prec", [bfm.PREC_FP64, bfm.PREC_FP32])
def test_near_field_shapes_agree(cluster, prec):
    """The symmetric near field's work item shapes (p2p_shape 0..2: receivers
    per chunk and sources per piece) only regroup the same pair sums: FP64
    products agree to rounding, FP32 ones to FP32 rounding, and each matches
    the all-pairs product to the expansion bound."""
    cl, phi = cluster
    ys = []
    for shape in (0, 1, 2):
        sv = bfm.Solver(p=16, p_lo=16, p2p_shape=shape)
        sv.set_cluster(cl)
        ys.append(sv.matvec(1.0, phi, precision=prec))
        if shape == 0:
            yd = sv.matvec(1.0, phi, direct=True)
    tol = 1e-12 if prec == bfm.PREC_FP64 else 2e-6
    for y in ys[1:]:
        d = float(np.max(np.abs(y - ys[0])) / np.max(np.abs(ys[0])))
        print(f"precision {prec}: shape difference {d:.2e}, vs all pairs {rel(y, yd):.2e}")
        assert d < tol and rel(y, yd) < (3e-7 if prec == bfm.PREC_FP64 else 3e-6)
    with pytest.raises(bfm.BfmError):
        bfm.Solver(p2p_shape=3)
