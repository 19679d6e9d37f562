"""Near-field correction matrices: higher-order quadrature of the boundary
integrals near each collocation point (Section 3.9, where the method's
nodal rule ns1 is combined with sparse "correction matrices" - the
difference between the BEM matrices of a high- and a low-order quadrature).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Reading (the paper names the idea and its source but fixes no rule):
* the boundary is the flat-triangle mesh with linear (hat) basis functions
  lambda_v; the exact collocation entries are
  L_iv = sum_{T ∋ v} int_T G(r_i, y) lambda_v(y) dS_y and
  M_iv = sum_{T ∋ v} int_T dG/dn_T(r_i, y) lambda_v(y) dS_y, n_T the flat
  triangle's unit normal; the nodal rule ns1 replaces each triangle's part
  by (A_T / 3) G(r_i, r_v) (and (A_T / 3) dG/dn_v(r_i, r_v) with the vertex
  normal n_v);
* near triangles of collocation point i: those with a vertex in {i} and its
  one-ring (the mesh neighbours of i);
* on a near triangle the integrals are taken with a conical Gauss product
  rule collapsed at the triangle's vertex nearest r_i (near-ties, squared
  distances within a relative 1e-9, go to the first in the triangle's
  vertex order):
  y = P0 + s (P1 - P0) + s t (P2 - P1), s, t in [0, 1] (Gauss-Legendre, ng
  points each), dS = 2 A_T s ds dt, barycentric (1 - s, s (1 - t), s t);
  when r_i is that vertex the factor s cancels the 1/|r_i - y| singularity
  and the double-layer integrand vanishes (r_i - y lies in the triangle's
  plane);
* the correction of entry (i, v), v != i, is the sum over the near
  triangles T ∋ v of [rule - nodal share]; the diagonal entries follow from
  the same identities as the nodal scheme, applied to the corrected
  off-diagonal entries (s3: M_ii = -1/2 - sum_j M_ij; s5: L_ii =
  n_i . [sum_j M_ij (r_j - r_i) - sum_j L_ij n_j]; eq3_1: b_i = -phi_i +
  sum_j M_ij (phi_j - phi_i)), so every diagonal correction is a sum over
  the row of the corrections.
"""
from __future__ import annotations

import numpy as np

from . import core

FOUR_PI = 4.0 * np.pi


def one_rings(tri, nv):
    """Sorted mesh neighbours of every vertex."""
    nb = [set() for _ in range(nv)]
    for a, b, c in np.asarray(tri):
        nb[a].update((b, c))
        nb[b].update((a, c))
        nb[c].update((a, b))
    return [np.array(sorted(x), dtype=np.int64) for x in nb]


def near_triangles(tri, nv):
    """Triangles with a vertex in {i} or the one-ring of i, sorted, per vertex."""
    tri = np.asarray(tri)
    vt = [[] for _ in range(nv)]
    for k, (a, b, c) in enumerate(tri):
        vt[a].append(k)
        vt[b].append(k)
        vt[c].append(k)
    rings = one_rings(tri, nv)
    out = []
    for i in range(nv):
        ts = set(vt[i])
        for j in rings[i]:
            ts.update(vt[j])
        out.append(np.array(sorted(ts), dtype=np.int64))
    return out


def conical_rule(ng):
    """Nodes (s, t) and weights of the Gauss-Legendre product rule on [0, 1]^2."""
    x, w = np.polynomial.legendre.leggauss(ng)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    s, t = np.meshgrid(x, x, indexing="ij")
    ww = np.outer(w, w)
    return s.ravel(), t.ravel(), ww.ravel()


def triangle_integrals(ri, P, nT, ng=8):
    """The three hat-weighted integrals of G and dG/dn_T over the triangle
    P[0], P[1], P[2] seen from r_i, collapsed at P[0] (the caller puts the
    vertex nearest r_i first). Returns (IL[3], IM[3])."""
    s, t, w = conical_rule(ng)
    P0, P1, P2 = P
    e1, e2 = P1 - P0, P2 - P1
    twoA = np.linalg.norm(np.cross(P1 - P0, P2 - P0))
    lam = np.stack([1.0 - s, s * (1.0 - t), s * t])
    if np.array_equal(ri, P0):
        d = e1[None, :] + t[:, None] * e2[None, :]  # (y - r_i) / s
        g = twoA / (FOUR_PI * np.linalg.norm(d, axis=1))  # G dS / (ds dt): the s cancels
        return lam @ (w * g), np.zeros(3)
    y = P0[None, :] + s[:, None] * e1[None, :] + (s * t)[:, None] * e2[None, :]
    dv = ri[None, :] - y
    r = np.linalg.norm(dv, axis=1)
    jac = twoA * s
    g = jac / (FOUR_PI * r)
    dg = jac * (dv @ nT) / (FOUR_PI * r ** 3)
    return lam @ (w * g), lam @ (w * dg)


def corrections(xyz, tri, s=None, n=None, rows=None, ng=8):
    """Correction entries of rows i (all by default), as a dict
    {i: (cols, CL, CM)} with cols the sorted j != i that any near triangle
    of i touches."""
    xyz = np.asarray(xyz, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.int64)
    nv = xyz.shape[0]
    if s is None or n is None:
        s, n, _ = core.geometry(xyz, tri)
    near = near_triangles(tri, nv)
    rows = range(nv) if rows is None else rows
    out = {}
    for i in rows:
        ri = xyz[i]
        acc = {}
        for k in near[i]:
            v = tri[k]
            P = xyz[v]
            nT = np.cross(P[1] - P[0], P[2] - P[0])
            area = 0.5 * np.linalg.norm(nT)
            nT = nT / (2.0 * area)
            # collapse at the vertex nearest r_i (r_i itself when it is one);
            # squared distances within a relative 1e-9 of the least count as
            # a tie, which goes to the first of them in the triangle's order
            d2 = ((P - ri[None, :]) ** 2).sum(axis=1)
            first = int(np.nonzero(d2 <= d2.min() * (1.0 + 1e-9))[0][0])
            order = [first, (first + 1) % 3, (first + 2) % 3]
            IL, IM = triangle_integrals(ri, P[order], nT, ng)
            for q in range(3):
                vv = int(v[order[q]])
                if vv == i:
                    continue
                dv = ri - xyz[vv]
                r = np.linalg.norm(dv)
                nodal_l = area / 3.0 / (FOUR_PI * r)
                nodal_m = area / 3.0 * (dv @ n[vv]) / (FOUR_PI * r ** 3)
                cl, cm = acc.get(vv, (0.0, 0.0))
                acc[vv] = (cl + IL[q] - nodal_l, cm + IM[q] - nodal_m)
        cols = np.array(sorted(acc), dtype=np.int64)
        out[i] = (cols, np.array([acc[j][0] for j in cols]), np.array([acc[j][1] for j in cols]))
    return out


def corrected_diagonals(xyz, n, phi, corr, Mii, Lii, b=None):
    """The diagonal entries and right-hand side of the corrected system, rows
    in the order of `corr`, from the nodal ones: M_ii - sum_j CM_ij,
    L_ii + n_i . [sum_j CM_ij (r_j - r_i) - sum_j CL_ij n_j],
    b_i + sum_j CM_ij (phi_j - phi_i)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    rows = list(corr)
    M2, L2 = np.array(Mii, dtype=np.float64).copy(), np.array(Lii, dtype=np.float64).copy()
    b2 = None if b is None else np.array(b, dtype=np.float64).copy()
    for k, i in enumerate(rows):
        cols, CL, CM = corr[i]
        M2[k] -= CM.sum()
        L2[k] += n[i] @ ((CM[:, None] * (xyz[cols] - xyz[i][None, :])).sum(axis=0) - (CL[:, None] * n[cols]).sum(axis=0))
        if b2 is not None:
            b2[k] += CM @ (phi[cols] - phi[i])
    return M2, L2, b2


def apply(corr, f, x, g=0.0, y=None, rows=None):
    """sum_j (f CL_ij x_j + g CM_ij y_j) for the rows of `corr` (or `rows`)."""
    rows = list(corr) if rows is None else rows
    out = np.zeros(len(rows))
    for k, i in enumerate(rows):
        cols, CL, CM = corr[i]
        if f != 0.0:
            out[k] += f * (CL @ x[cols])
        if g != 0.0:
            out[k] += g * (CM @ y[cols])
    return out


def solve(xyz, tri, phi, tol=1e-12, restart=50, maxit=2000, ng=8):
    """L q = b with the corrected matrices (all rows; small meshes)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    s, n, _ = core.geometry(xyz, tri)
    d = core.sums(xyz, s, n, phi)
    Mii, Lii, _ = core.diagonals(xyz, s, n, sm=d)
    b = core.rhs(phi, d["B"])
    corr = corrections(xyz, tri, s, n, ng=ng)
    M2, L2, b2 = corrected_diagonals(xyz, n, phi, corr, Mii, Lii, b)

    def mv(v):
        return core.offdiag_mvp(xyz, s, n, 1.0, v) + apply(corr, 1.0, v) + L2 * v
    q, info = core.gmres(mv, b2, tol=tol, restart=restart, maxit=maxit)
    info.update(Mii=M2, Lii=L2, b=b2, corr=corr)
    return q, info
