"""Toroidal (genus-1) bubbles in the oracle (Section 3.7, spherical7; the
boundary-element system itself does not depend on the genus). Pins: the
template mesh is closed, outward and of Euler characteristic 0; polyhedral
volumes converge to 2 pi^2 R a^2; Gauss's identity sum_j M_ij -> -1/2 and the
exact Neumann data of a point source inside the tube (the oracle's solve)
converge under refinement; the toroidal filter is an orthogonal projector of
rank (p_f + 1)^2 that keeps trigonometric polynomials of degree <= p_f/2 in
each angle (the torus coordinates among them) and is the identity on a
(p_f + 1) x (p_f + 1) grid; the paraboloid curvature matches the torus's mean
curvature in closed form.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import step as st
from paper_1905_01341_amd import workload as wl

A = wl.TORUS_TUBE


def test_template_is_closed_and_outward():
    v, f, ang = wl.torus(48, 16)
    edges = {}
    for t in f:
        for k in range(3):
            e = (int(t[k]), int(t[(k + 1) % 3]))
            edges[e] = edges.get(e, 0) + 1
    assert all(c == 1 for c in edges.values())
    assert all((b, a) in edges for a, b in edges)  # every edge twice, opposite directions
    assert len(v) - len(edges) // 2 + len(f) == 0  # genus 1
    c = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])
    cen = v[f].mean(axis=1)
    ph = np.arctan2(cen[:, 1], cen[:, 0])
    axis = np.stack([np.cos(ph), np.sin(ph), 0 * ph], axis=1)
    assert np.all(np.einsum("ij,ij->i", c, cen - axis) > 0)
    th, p = ang.T
    rho = 1.0 + A * np.cos(th)
    assert np.allclose(v, np.stack([rho * np.cos(p), rho * np.sin(p), A * np.sin(th)], axis=1))


def test_volume_converges():
    exact = 2.0 * math.pi ** 2 * A ** 2
    errs = []
    for n in (8, 16, 32):
        v, f, _ = wl.torus(3 * n, n)
        vol = st.volumes(v, f, [0, len(f)])[0]
        errs.append(abs(vol - exact) / exact)
    assert errs[2] < 1e-2 and errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs


def test_gauss_identity_on_torus():
    """sum_{j != i} M_ij -> -1/2 at every vertex of a closed surface."""
    errs = []
    for n in (8, 16):
        v, f, _ = wl.torus(3 * n, n)
        s, nrm, _ = oracle.geometry(v, f)
        sm = oracle.sums(v, s, nrm)["SM"]
        errs.append(np.max(np.abs(sm + 0.5)))
    assert errs[1] < 0.06 and errs[0] / errs[1] > 1.8, errs  # first order, as on spheres


def _source_field(v, ang, x0):
    """phi = 1/|r - x0| and its exact outward normal derivative."""
    th, p = ang.T
    n = np.stack([np.cos(th) * np.cos(p), np.cos(th) * np.sin(p), np.sin(th)], axis=1)
    d = v - x0
    r = np.linalg.norm(d, axis=1)
    return 1.0 / r, -np.einsum("ij,ij->i", d, n) / r ** 3


def test_exact_neumann_data_of_a_source_inside_the_tube():
    """A point source on the tube's centre circle (inside the gas) gives a
    potential harmonic in the liquid and vanishing at infinity: the solve
    must return its normal derivative, to the discretisation error, which
    falls at second order."""
    x0 = np.array([math.cos(0.3), math.sin(0.3), 0.05])
    errs = []
    for n in (8, 16):
        v, f, ang = wl.torus(3 * n, n)
        phi, q_exact = _source_field(v, ang, x0)
        q, info = oracle.solve(v, f, phi, method="lu")
        errs.append(np.max(np.abs(q - q_exact)) / np.max(np.abs(q_exact)))
    assert errs[1] < 0.03 and errs[0] / errs[1] > 3.0, errs


@pytest.mark.parametrize("pf", [2, 4, 8])
def test_torus_filter_is_a_projector(pf):
    v, f, ang = wl.torus(48, 16)
    F = st.filter_matrix_torus(ang, pf)
    assert np.allclose(F @ F, F, atol=1e-12)
    assert np.allclose(F, F.T, atol=1e-12)
    assert abs(np.trace(F) - (pf + 1) ** 2) < 1e-9
    th, p = ang.T
    h = pf // 2
    keep = np.cos(h * th) * np.sin(h * p) + np.sin(th) - 0.5 * np.cos(2 * p) * (pf >= 4)
    assert np.allclose(F @ keep, keep, atol=1e-12)
    assert np.allclose(F @ v, v, atol=1e-12)  # the torus is degree 1 in each angle
    cut = np.cos((h + 1) * th)  # one degree above the band: projected out
    assert np.max(np.abs(F @ cut)) < 1e-12


def test_torus_filter_identity_and_errors():
    pf = 4
    _, _, ang = wl.torus(pf + 1, pf + 1)
    assert np.allclose(st.filter_matrix_torus(ang, pf), np.eye((pf + 1) ** 2), atol=1e-12)
    with pytest.raises(ValueError):
        st.torus_basis(ang, 3)


def test_paraboloid_curvature_of_a_torus():
    """H = (1/a + cos theta / (1 + a cos theta)) / 2 (outward normal, the
    sphere's H = 1/R convention), to first order in the grid spacing: the
    five-neighbour stencil of this grid is not symmetric and the vertex
    normal is an area-weighted average (measured: 28%, 14%, 9% at 16, 32,
    48 cells around the tube, worst on the inner side)."""
    errs = []
    for n in (16, 32):
        v, f, ang = wl.torus(3 * n, n)
        s, nrm, _ = oracle.geometry(v, f)
        H = st.curvature(v, nrm, st.one_ring(f, len(v)))
        th = ang[:, 0]
        exact = 0.5 * (1.0 / A + np.cos(th) / (1.0 + A * np.cos(th)))
        errs.append(np.max(np.abs(H - exact) / exact))
    assert errs[1] < 0.15 and errs[0] / errs[1] > 1.8, errs
