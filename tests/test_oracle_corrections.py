"""Pins of the near-field correction oracle (oracle/corrections.py, Section
3.9's correction matrices) against what the mathematics fixes, computed by
routes that share nothing with its conical rule:

* the weakly singular self integral of a flat triangle (collocation point at
  a vertex) against its closed form in polar coordinates, h ln(sec + tan);
* the double-layer integral of a flat triangle against the solid angle it
  subtends (Van Oosterom and Strackee 1983);
* every hat-weighted integral against adaptive two-dimensional quadrature
  (scipy dblquad over the barycentric parametrisation);
* the assembled corrected matrices of a small closed mesh against a matrix
  built entry by entry from those brute-force integrals on the near
  triangles and the nodal shares on the rest;
* the pattern against its definition read off the edge graph.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import corrections as oc
from paper_1905_01341_amd import workload as wl

FOUR_PI = 4.0 * math.pi


def _tri(seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(3, 3))


def _brute(ri, P, nT, q, kind):
    """int_T lambda_q K dS by adaptive quadrature over (u, v), y = P0 + u (P1 -
    P0) + v (P2 - P0), lambda = (1 - u - v, u, v), dS = 2 A du dv; K = G or
    dG/dn_T with G = 1 / (4 pi |r - y|)."""
    P0, P1, P2 = P
    twoA = np.linalg.norm(np.cross(P1 - P0, P2 - P0))

    def f(v, u):
        y = P0 + u * (P1 - P0) + v * (P2 - P0)
        lam = (1.0 - u - v, u, v)[q]
        d = ri - y
        r = math.sqrt(d @ d)
        k = 1.0 / (FOUR_PI * r) if kind == "L" else (d @ nT) / (FOUR_PI * r ** 3)
        return lam * k * twoA

    val, _ = integrate.dblquad(f, 0.0, 1.0, 0.0, lambda u: 1.0 - u, epsabs=1e-13, epsrel=1e-12)
    return val


def _normal(P):
    n = np.cross(P[1] - P[0], P[2] - P[0])
    return n / np.linalg.norm(n)


def test_conical_rule_weights():
    """The product rule on [0, 1]^2 integrates s^a t^b exactly up to degree
    2 ng - 1 in each variable."""
    s, t, w = oc.conical_rule(8)
    for a in range(16):
        for b in (0, 3, 15):
            assert abs(w @ (s ** a * t ** b) - 1.0 / ((a + 1) * (b + 1))) < 1e-14


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_self_integral_closed_form(seed):
    """r_i at P0: int_T dS / |y - P0| = h [ln(sec phi + tan phi)] between the
    angles phi1, phi2 of the edges P0P1, P0P2 from the foot of the
    perpendicular (distance h) to the opposite edge. The double layer
    vanishes there (r_i - y lies in the plane)."""
    P = _tri(seed)
    a, b = P[1] - P[0], P[2] - P[0]
    e = b - a
    foot = a - (a @ e) / (e @ e) * e  # P0 -> foot of the perpendicular
    h = np.linalg.norm(foot)
    ang = [math.copysign(math.acos(min(1.0, (x @ foot) / (np.linalg.norm(x) * h))), (x - foot) @ e)
           for x in (a, b)]
    F = [math.log(1.0 / math.cos(p) + math.tan(p)) for p in ang]
    exact = h * (F[1] - F[0]) / FOUR_PI
    for ng, tol in ((8, 1e-5), (24, 1e-11)):
        IL, IM = oc.triangle_integrals(P[0].copy(), P, _normal(P), ng=ng)
        assert abs(IL.sum() - exact) < tol * exact, ng
        assert np.all(IM == 0.0)
    for q in range(3):  # ng = 24 against the adaptive rule
        assert abs(IL[q] - _brute(P[0], P, _normal(P), q, "L")) < 1e-9 * exact


def _solid_angle(r, P):
    a, b, c = (x - r for x in P)
    la, lb, lc = (np.linalg.norm(x) for x in (a, b, c))
    num = a @ np.cross(b, c)
    den = la * lb * lc + (a @ b) * lc + (a @ c) * lb + (b @ c) * la
    return 2.0 * math.atan2(num, den)


@pytest.mark.parametrize("seed", [4, 5, 6])
@pytest.mark.parametrize("height", [0.3, 1.0])
def test_double_layer_is_solid_angle(seed, height):
    """sum_q int lambda_q dG/dn_T = -Omega / (4 pi), Omega the signed solid
    angle of the triangle seen from r_i (van Oosterom-Strackee, negative when
    n_T points towards r_i). ng = 40 reaches it at 0.3 side lengths above
    the triangle, ng = 8 at one side length; closer above the interior the
    rule collapsed at a vertex does not resolve the peak (a collocation point
    is a vertex, so its near triangles are seen from their edges)."""
    P = _tri(seed)
    nT = _normal(P)
    cen = P.mean(axis=0)
    ri = cen + height * nT + 0.2 * (P[1] - P[0])
    d2 = ((P - ri) ** 2).sum(axis=1)
    k = int(np.argmin(d2))
    order = [k, (k + 1) % 3, (k + 2) % 3]
    om = _solid_angle(ri, P)
    for ng, tol in ((40, 1e-9), (8, 1e-5 if height >= 1.0 else None)):
        if tol is None:
            continue
        _, IM = oc.triangle_integrals(ri, P[order], nT, ng=ng)
        assert abs(IM.sum() + om / FOUR_PI) < tol * max(abs(om) / FOUR_PI, 1e-3), (ng, height)


@pytest.mark.parametrize("seed", [7, 8])
def test_hat_weighted_integrals_brute_force(seed):
    """Each of the three hat-weighted integrals of G and dG/dn_T, collapsed at
    the vertex nearest r_i, against adaptive quadrature (point at about a
    side's length from the triangle)."""
    P = _tri(seed)
    nT = _normal(P)
    ri = P.mean(axis=0) + 0.4 * nT + 0.6 * (P[2] - P[1])
    d2 = ((P - ri) ** 2).sum(axis=1)
    k = int(np.argmin(d2))
    order = [k, (k + 1) % 3, (k + 2) % 3]
    IL, IM = oc.triangle_integrals(ri, P[order], nT, ng=16)
    for q in range(3):
        bl = _brute(ri, P, nT, order[q], "L")
        bm = _brute(ri, P, nT, order[q], "M")
        assert abs(IL[q] - bl) < 1e-9 * abs(IL).max(), q
        assert abs(IM[q] - bm) < 1e-9 * abs(IM).max(), q


def _mesh():
    xyz, tri = wl.icosphere(1)
    rng = np.random.default_rng(11)
    xyz = xyz * (1.0 + 0.05 * rng.uniform(-1.0, 1.0, size=(len(xyz), 1)))
    return xyz, tri


def test_pattern_from_edge_graph():
    """Near triangles of i: those with a vertex equal or adjacent to i (edge
    graph); the row's columns: every other vertex of them."""
    xyz, tri = _mesh()
    nv = len(xyz)
    adj = np.zeros((nv, nv), bool)
    for t in tri:
        for a in range(3):
            adj[t[a], t[(a + 1) % 3]] = adj[t[(a + 1) % 3], t[a]] = True
    near = oc.near_triangles(tri, nv)
    corr = oc.corrections(xyz, tri, rows=[0, 5, 17])
    for i in range(nv):
        ball = adj[i] | (np.arange(nv) == i)
        want = [k for k, t in enumerate(tri) if ball[t].any()]
        assert list(near[i]) == want
    for i, (cols, _, _) in corr.items():
        want = sorted({int(v) for k in near[i] for v in tri[k]} - {i})
        assert list(cols) == want


def test_corrected_matrix_brute_force():
    """Nodal matrix + corrections, rows of a perturbed icosphere (42
    vertices), against entries assembled independently: on every near
    triangle T of i the brute-force integral of lambda_j K, on every other
    triangle the nodal share A_T / 3 K(r_i, r_j) (vertex normal n_j for the
    double layer). ng = 20 makes the rule's own error negligible."""
    xyz, tri = _mesh()
    nv = len(xyz)
    s, n, area = oracle.geometry(xyz, tri)
    L0, M0 = oracle.dense_offdiag(xyz, s, n)
    rows = [3, 20]
    corr = oc.corrections(xyz, tri, s, n, rows=rows, ng=20)
    near = oc.near_triangles(tri, nv)
    for i in rows:
        Lb = np.zeros(nv)
        Mb = np.zeros(nv)
        for k, t in enumerate(tri):
            P = xyz[t]
            nT = _normal(P)
            for q in range(3):
                j = int(t[q])
                if j == i:
                    continue
                if k in set(near[i].tolist()):
                    Lb[j] += _brute(xyz[i], P, nT, q, "L")
                    Mb[j] += _brute(xyz[i], P, nT, q, "M")
                else:
                    d = xyz[i] - xyz[j]
                    r = np.linalg.norm(d)
                    Lb[j] += area[k] / 3.0 / (FOUR_PI * r)
                    Mb[j] += area[k] / 3.0 * (d @ n[j]) / (FOUR_PI * r ** 3)
        cols, CL, CM = corr[i]
        Lc, Mc = L0[i].copy(), M0[i].copy()
        Lc[cols] += CL
        Mc[cols] += CM
        Lc[i] = Mc[i] = 0.0
        assert np.max(np.abs(Lc - Lb)) < 1e-9 * np.max(np.abs(Lb)), i
        assert np.max(np.abs(Mc - Mb)) < 1e-9 * np.max(np.abs(Mb)), i
        # the corrections are not small: the nodal rule is off by O(1) near i
        assert np.max(np.abs(CL)) > 0.05 * np.max(np.abs(L0[i]))


def test_corrected_diagonals_are_row_identities():
    """With the corrected off-diagonal entries, M_ii = -1/2 - sum_j M_ij (s3),
    L_ii = n_i . [sum_j M_ij (r_j - r_i) - sum_j L_ij n_j] (s5) and b_i =
    -phi_i + sum_j M_ij (phi_j - phi_i) (eq3_1), evaluated on the dense
    corrected rows."""
    xyz, tri = _mesh()
    nv = len(xyz)
    s, n, _ = oracle.geometry(xyz, tri)
    L0, M0 = oracle.dense_offdiag(xyz, s, n)
    phi = np.cos(np.arange(nv) * 0.7)
    Mii, Lii, _ = oracle.diagonals(xyz, s, n)
    b = oracle.rhs(phi, oracle.sums(xyz, s, n, phi)["B"])
    corr = oc.corrections(xyz, tri, s, n)
    M2, L2, b2 = oc.corrected_diagonals(xyz, n, phi, corr, Mii, Lii, b)
    for i in range(nv):
        cols, CL, CM = corr[i]
        Lr, Mr = L0[i].copy(), M0[i].copy()
        Lr[cols] += CL
        Mr[cols] += CM
        Lr[i] = Mr[i] = 0.0
        assert abs(M2[i] - (-0.5 - Mr.sum())) < 1e-13
        want = n[i] @ ((Mr[:, None] * (xyz - xyz[i])).sum(axis=0) - (Lr[:, None] * n).sum(axis=0))
        assert abs(L2[i] - want) < 1e-13
        assert abs(b2[i] - (-phi[i] + Mr @ (phi - phi[i]))) < 1e-13


def test_corrected_solve_on_a_sphere():
    """Sphere, phi = 1: the corrected system's solution q = -phi (flux of
    1/r) to the discretisation error, which the corrections do not reduce
    below the nodal rule's at these sizes (they fix the near entries but the
    error is dominated by the flat-triangle geometry)."""
    xyz, tri = wl.icosphere(2)
    phi = np.ones(len(xyz))
    q, info = oc.solve(xyz, tri, phi, tol=1e-12)
    q0, _ = oracle.solve(xyz, tri, phi, tol=1e-12)
    e = np.max(np.abs(q + 1.0))
    e0 = np.max(np.abs(q0 + 1.0))
    assert e < 0.05 and e0 < 0.05
    assert e < 3.0 * e0
