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
    assert abs(r["lmax"] - lmax0) <= 1 and r["m2l_shape"] in (0, 1, 2, 3)
    assert r["candidates"] >= 6 and r["mvp_ms"] > 0
    assert sv.tree_stats()["lmax"] == r["lmax"]
    q, info = sv.solve(phi)
    ref = bfm.Solver(p=20, gmres_tol=1e-10, precond=bfm.PRECOND_SH_COARSE)
    ref.set_cluster(cl)
    q20, _ = ref.solve(phi)
    assert info["converged"] and rel(q, q20) < 1e-6
