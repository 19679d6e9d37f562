"""FP64 reference of one explicit time step of the bubble dynamics
(test infrastructure).

TEST INFRASTRUCTURE ONLY (see the package docstring). Follows the paper:

* shape filter of bandwidth p_f (Section 3.7, eq3_22-eq3_25, spherical6):
  F = G (G^T G)^{-1} G^T per bubble, G the real harmonics of degree
  0..p_f-1 at the template directions of the bubble's vertices; applied to
  r and phi before the right-hand side and to dr/dt and dphi/dt after it;
  for toroidal bubbles (genus 1, spherical7) G is the real trigonometric
  basis of the two angles of each vertex on the template torus, degrees
  0..p_f/2 in each (p_f even, (p_f + 1)^2 columns);
* geometry (Section 3.2, ns1) and bubble volumes by the divergence theorem
  over the flat triangles, V = sum r1 . (r2 x r3) / 6 (about the bubble's
  own first vertex);
* mean curvature by the fitted paraboloid (Section 3.5, parab1/parab2):
  five one-ring neighbours, local frame with z along n_j, 5 x 5 solve,
  H = -B3 - B5;
* tangential velocity from Stokes' theorem on each triangle (eq3_10) and
  the area-weighted vertex average (eq3_11);
* the solve for q (Section 3.1, eq3_2) by dense LU (core.solve);
* u = v + alpha v_t (eq3_13), dr/dt = u (eq3_14),
  dphi/dt = (alpha v_t + v/2) . v - (p_g - 2 sigma H)/rho + g . r + p_inf(t)/rho
  (eq3_15) with the polytropic gas pressure p_g = p_g0 (V0/V)^kappa and
  p_g0 = p0 + 2 sigma / a0 (eq2_8);
* fourth-order Runge-Kutta for the first five steps, then the sixth-order
  Adams-Bashforth method (Section 3.6); the Adams-Bashforth weights are
  derived here from the integrated Lagrange basis with exact fractions.

Readings: the five neighbours are the first five of the vertex's one-ring in
counter-clockwise order (seen from outside) starting at the neighbour with
the lowest index, and the local x axis is the tangential projection of the
edge to that first neighbour; V0 and a0 = (3 V0 / 4 pi)^(1/3) come from the
filtered initial shape; p_inf(t) = p0 + sign * P_a * sin(2 pi t / T) (the
paper's eq2_6 has sign -1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from fractions import Fraction

import numpy as np

from . import core
from .learned import real_sh


@dataclass
class Physics:
    rho: float = 1.0
    p0: float = 1.0
    sigma: float = 0.0
    kappa: float = 1.4
    pa: float = 0.0
    period: float = 0.0
    forcing_sign: float = -1.0
    g: tuple = (0.0, 0.0, 0.0)
    alpha: float = -1.0
    filter_degree: int = 0

    def p_inf(self, t):
        if self.period <= 0.0 or self.pa == 0.0:
            return self.p0
        return self.p0 + self.forcing_sign * self.pa * math.sin(2 * math.pi * t / self.period)


def filter_matrix(dirs, pf):
    """F = G (G^T G)^{-1} G^T for harmonics of degree 0..pf-1 (eq3_25)."""
    G = real_sh(pf - 1, dirs)
    return G @ np.linalg.solve(G.T @ G, G.T)


def torus_basis(angles, pf):
    """Real trigonometric basis of bandwidth pf (pf even) at (theta, phi):
    every product of {1, cos k theta, sin k theta : k = 1..pf/2} with the
    same set in phi - the real form of e^{i(n theta + m phi)}, |n|, |m| <=
    pf/2 (spherical7). [nd, (pf + 1)^2]."""
    if pf % 2:
        raise ValueError("the toroidal filter needs an even bandwidth")
    th, ph = np.asarray(angles, dtype=np.float64).T

    def one(x):
        cols = [np.ones_like(x)]
        for k in range(1, pf // 2 + 1):
            cols += [np.cos(k * x), np.sin(k * x)]
        return np.stack(cols, axis=1)
    A, B = one(th), one(ph)
    return (A[:, :, None] * B[:, None, :]).reshape(len(th), -1)


def filter_matrix_torus(angles, pf):
    """F = G (G^T G)^{-1} G^T with the toroidal basis (spherical7)."""
    G = torus_basis(angles, pf)
    return G @ np.linalg.solve(G.T @ G, G.T)


def apply_filter(F, values, nb, nd):
    """Filter per bubble: values [nb * nd, ...] -> same shape."""
    v = np.asarray(values, dtype=np.float64)
    shp = v.shape
    v = v.reshape(nb, nd, -1)
    return np.einsum("ij,bjk->bik", F, v).reshape(shp)


def volumes(xyz, tri, tri_off):
    """Per-bubble volume of the closed polyhedron (divergence theorem),
    V = sum (r1 - o) . ((r2 - o) x (r3 - o)) / 6, which is the same for any
    origin o of a closed surface; o = the first vertex of the bubble's first
    triangle keeps the terms at the bubble's own scale."""
    r = np.asarray(xyz, dtype=np.float64)
    t = np.asarray(tri)
    out = []
    for b in range(len(tri_off) - 1):
        tb = t[tri_off[b]:tri_off[b + 1]]
        o = r[tb[0, 0]]
        a, bb, c = r[tb[:, 0]] - o, r[tb[:, 1]] - o, r[tb[:, 2]] - o
        out.append(np.einsum("ij,ij->i", a, np.cross(bb, c)).sum() / 6.0)
    return np.array(out)


def one_ring(tri, nv):
    """Neighbours of every vertex in counter-clockwise order seen from
    outside (triangles (a, b, c) are counter-clockwise from outside, so
    around a the edge b -> c advances counter-clockwise), starting at the
    neighbour with the lowest index."""
    nxt = [dict() for _ in range(nv)]
    for a, b, c in np.asarray(tri):
        nxt[a][b] = c
        nxt[b][c] = a
        nxt[c][a] = b
    rings = []
    for j in range(nv):
        start = min(nxt[j])
        ring = [start]
        while True:
            k = nxt[j][ring[-1]]
            if k == start:
                break
            ring.append(k)
        assert len(ring) == len(nxt[j]), "vertex one-ring is not a single cycle"
        rings.append(ring)
    return rings


def curvature(xyz, n, rings):
    """Mean curvature H_j from the paraboloid through five neighbours."""
    r = np.asarray(xyz, dtype=np.float64)
    H = np.empty(r.shape[0])
    for j, ring in enumerate(rings):
        nb5 = ring[:5]
        ez = n[j]
        e = r[nb5[0]] - r[j]
        ex = e - np.dot(e, ez) * ez
        ex /= np.linalg.norm(ex)
        ey = np.cross(ez, ex)
        Q = np.empty((5, 5))
        zr = np.empty(5)
        for l, k in enumerate(nb5):
            d = r[k] - r[j]
            x, y, z = np.dot(d, ex), np.dot(d, ey), np.dot(d, ez)
            Q[l] = (x, y, x * x, x * y, y * y)
            zr[l] = z
        B = np.linalg.solve(Q, zr)
        H[j] = -B[2] - B[4]
    return H


def tangential_velocity(xyz, tri, phi, s, n, area):
    """v_t at every vertex (eq3_10, eq3_11)."""
    r = np.asarray(xyz, dtype=np.float64)
    t = np.asarray(tri)
    p = np.asarray(phi, dtype=np.float64)
    r1, r2, r3 = r[t[:, 0]], r[t[:, 1]], r[t[:, 2]]
    nxv_k = ((r2 - r3) * p[t[:, 0], None] + (r3 - r1) * p[t[:, 1], None]
             + (r1 - r2) * p[t[:, 2], None]) / (2.0 * area[:, None])
    acc = np.zeros_like(r)
    for c in range(3):
        np.add.at(acc, t[:, c], nxv_k * area[:, None])
    nxv = acc / (3.0 * s[:, None])
    return np.cross(nxv, n)


@dataclass
class Mesh:
    tri: np.ndarray
    vtx_off: np.ndarray
    tri_off: np.ndarray
    dirs: np.ndarray          # template directions [nd, 3] (spheres) or angles [nd, 2] (tori)
    nb: int
    nd: int
    rings: list = field(default=None)
    F: np.ndarray = field(default=None)


def make_mesh(tri, vtx_off, tri_off, dirs, pf, torus=False):
    """Connectivity, one-rings and the filter of bandwidth pf; dirs are the
    template's unit directions [nd, 3], or with torus its angles [nd, 2]."""
    nb = len(vtx_off) - 1
    nd = int(vtx_off[1] - vtx_off[0])
    nv = nb * nd
    m = Mesh(np.asarray(tri), np.asarray(vtx_off), np.asarray(tri_off), np.asarray(dirs), nb, nd)
    m.rings = one_ring(m.tri, nv)
    if pf > 0:
        m.F = filter_matrix_torus(dirs, pf) if torus else filter_matrix(dirs, pf)
    return m


def rhs(mesh, phys, V0, pg0, t, xyz, phi):
    """Right-hand side of eq3_14/eq3_15. Returns (dxyz, dphi, q, H) with the
    filter applied to inputs and outputs when phys.filter_degree > 0."""
    nb, nd = mesh.nb, mesh.nd
    if mesh.F is not None:
        xyz = apply_filter(mesh.F, xyz, nb, nd)
        phi = apply_filter(mesh.F, phi, nb, nd)
    s, n, area = core.geometry(xyz, mesh.tri)
    q, _ = core.solve(xyz, mesh.tri, phi, method="lu")
    H = curvature(xyz, n, mesh.rings)
    vt = tangential_velocity(xyz, mesh.tri, phi, s, n, area)
    v = n * q[:, None] + vt
    u = v + phys.alpha * vt
    V = volumes(xyz, mesh.tri, mesh.tri_off)
    pg = np.repeat(pg0 * (V0 / V) ** phys.kappa, nd)
    g = np.asarray(phys.g, dtype=np.float64)
    dphi = (np.einsum("ij,ij->i", phys.alpha * vt + 0.5 * v, v) - (pg - 2.0 * phys.sigma * H) / phys.rho
            + xyz @ g + phys.p_inf(t) / phys.rho)
    dxyz = u
    if mesh.F is not None:
        dxyz = apply_filter(mesh.F, dxyz, nb, nd)
        dphi = apply_filter(mesh.F, dphi, nb, nd)
    return dxyz, dphi, q, H


def adams_bashforth_weights(order):
    """Weights b_k (k = 0 newest .. order-1 oldest) of the explicit Adams
    method: y_{n+1} = y_n + dt sum_k b_k f_{n-k}, from the integral over
    [0, 1] of the Lagrange basis on the nodes 0, -1, ..., -(order-1)."""
    nodes = [Fraction(-k) for k in range(order)]
    w = []
    for k in range(order):
        # polynomial prod_{i != k} (x - x_i) / (x_k - x_i), coefficients low -> high
        coef = [Fraction(1)]
        den = Fraction(1)
        for i in range(order):
            if i == k:
                continue
            coef = [Fraction(0)] + coef
            for d in range(len(coef) - 1):
                coef[d] -= nodes[i] * coef[d + 1]
            den *= nodes[k] - nodes[i]
        w.append(sum(c / (d + 1) for d, c in enumerate(coef)) / den)
    return w


def initial_gas(mesh, phys, xyz):
    """V0 per bubble (of the filtered initial shape) and p_g0 = p0 + 2 sigma / a0."""
    x = apply_filter(mesh.F, xyz, mesh.nb, mesh.nd) if mesh.F is not None else np.asarray(xyz, float)
    V0 = volumes(x, mesh.tri, mesh.tri_off)
    a0 = (3.0 * V0 / (4.0 * math.pi)) ** (1.0 / 3.0)
    return V0, phys.p0 + 2.0 * phys.sigma / a0


class Integrator:
    """RK4 for the first five steps, sixth-order Adams-Bashforth after."""

    def __init__(self, mesh, phys, xyz, phi, t0=0.0):
        self.mesh, self.phys = mesh, phys
        self.xyz = np.array(xyz, dtype=np.float64)
        self.phi = np.array(phi, dtype=np.float64)
        self.t = float(t0)
        self.V0, self.pg0 = initial_gas(mesh, phys, self.xyz)
        self.hist = []  # (dxyz, dphi) at past step starts, newest first
        self.steps = 0
        self.ab = [float(w) for w in adams_bashforth_weights(6)]

    def f(self, t, xyz, phi):
        dx, dp, _, _ = rhs(self.mesh, self.phys, self.V0, self.pg0, t, xyz, phi)
        return dx, dp

    def step(self, dt):
        if self.steps < 5:
            k1 = self.f(self.t, self.xyz, self.phi)
            self.hist.insert(0, k1)
            k2 = self.f(self.t + dt / 2, self.xyz + dt / 2 * k1[0], self.phi + dt / 2 * k1[1])
            k3 = self.f(self.t + dt / 2, self.xyz + dt / 2 * k2[0], self.phi + dt / 2 * k2[1])
            k4 = self.f(self.t + dt, self.xyz + dt * k3[0], self.phi + dt * k3[1])
            self.xyz = self.xyz + dt / 6 * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0])
            self.phi = self.phi + dt / 6 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1])
        else:
            self.hist.insert(0, self.f(self.t, self.xyz, self.phi))
            self.xyz = self.xyz + dt * sum(w * h[0] for w, h in zip(self.ab, self.hist))
            self.phi = self.phi + dt * sum(w * h[1] for w, h in zip(self.ab, self.hist))
        del self.hist[6:]
        self.t += dt
        self.steps += 1
