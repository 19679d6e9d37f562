"""FP64 reference for the learned initial guess (test infrastructure).

TEST INFRASTRUCTURE ONLY (see the package docstring). The learned guess is
not part of the paper: the paper starts GMRES from the previous time step's
q (Section 3.6). What is defined here is what the GPU computes for it:

* real spherical harmonics Y_k (k = n^2 for order 0; n^2 + 2m - 1 and n^2 + 2m
  for the cos(m lon) and sin(m lon) parts of order m = 1..n), orthonormal on
  the unit sphere, without the Condon-Shortley phase;
* per bubble b (vertices on a common template of unit directions d_i, as
  for the paper's shape filter, Section 3.7): centre c_b (vertex mean),
  equivalent radius a_b = sqrt(area_b / 4 pi) with area_b the sum of the
  vertex weights s_i, and the weighted least-squares projection
  G+ = (G^T W G)^{-1} G^T W onto degrees <= 8 (G_ik = Y_k(d_i), W = areas of
  the template vertices on the unit sphere, one third of every incident
  triangle);
* features [G+ (|r_i - c_b| / a_b) (81) | G+ phi (81) | offsets of the 4
  nearest other centres / a_b (12)], target G+ (a_b q) (81), and the guess
  q_i = (G c)_i / a_b from predicted coefficients c.

``bf16`` rounds to bfloat16 (round to nearest, ties to even, through FP32):
the MLP reference applies it where the GPU kernels store BF16 operands.
"""
from __future__ import annotations

import math

import numpy as np

DEGREE = 8
NC = (DEGREE + 1) ** 2
N_IN = 2 * NC + 12


def legendre_table(nmax, t):
    """Associated Legendre P_n^m(t), no Condon-Shortley phase, for
    0 <= m <= n <= nmax; returns a dict (n, m) -> array (textbook
    recurrences: P_m^m = (2m-1)!! (1-t^2)^(m/2), P_{m+1}^m = (2m+1) t P_m^m,
    (n-m) P_n^m = (2n-1) t P_{n-1}^m - (n+m-1) P_{n-2}^m)."""
    t = np.asarray(t, dtype=np.float64)
    s = np.sqrt(np.maximum(0.0, 1.0 - t * t))
    P = {}
    pmm = np.ones_like(t)
    for m in range(nmax + 1):
        if m > 0:
            pmm = pmm * (2 * m - 1) * s
        P[(m, m)] = pmm
        if m + 1 <= nmax:
            P[(m + 1, m)] = (2 * m + 1) * t * pmm
        for n in range(m + 2, nmax + 1):
            P[(n, m)] = ((2 * n - 1) * t * P[(n - 1, m)] - (n + m - 1) * P[(n - 2, m)]) / (n - m)
    return P


def real_sh(nmax, dirs):
    """Orthonormal real harmonics at unit vectors dirs [n, 3] -> [n, (nmax+1)^2]."""
    d = np.asarray(dirs, dtype=np.float64)
    t = d[:, 2]
    lon = np.arctan2(d[:, 1], d[:, 0])
    P = legendre_table(nmax, t)
    out = np.zeros((d.shape[0], (nmax + 1) ** 2))
    for n in range(nmax + 1):
        for m in range(n + 1):
            norm = math.sqrt((2 * n + 1) / (4 * math.pi) * math.factorial(n - m) / math.factorial(n + m))
            if m == 0:
                out[:, n * n] = norm * P[(n, 0)]
            else:
                out[:, n * n + 2 * m - 1] = math.sqrt(2.0) * norm * P[(n, m)] * np.cos(m * lon)
                out[:, n * n + 2 * m] = math.sqrt(2.0) * norm * P[(n, m)] * np.sin(m * lon)
    return out


def template_weights(dirs, tri0):
    """One third of the area of every incident flat triangle on the unit directions."""
    d = np.asarray(dirs, dtype=np.float64)
    tri0 = np.asarray(tri0)
    w = np.zeros(d.shape[0])
    for a, b, c in tri0:
        area = 0.5 * np.linalg.norm(np.cross(d[b] - d[a], d[c] - d[a]))
        w[a] += area / 3
        w[b] += area / 3
        w[c] += area / 3
    return w


def projector(dirs, tri0, nmax=DEGREE):
    """(G [nd, nc], G+ [nc, nd]) with G+ = (G^T W G)^{-1} G^T W."""
    G = real_sh(nmax, dirs)
    w = template_weights(dirs, tri0)
    S = G.T @ (w[:, None] * G)
    Gp = np.linalg.solve(S, G.T * w[None, :])
    return G, Gp


def bubble_frames(xyz, s, nb, nd):
    """Centres (vertex means) [nb, 3] and radii sqrt(sum s / 4 pi) [nb]."""
    X = np.asarray(xyz, dtype=np.float64).reshape(nb, nd, 3)
    cen = X.mean(axis=1)
    rad = np.sqrt(np.asarray(s, dtype=np.float64).reshape(nb, nd).sum(axis=1) / (4 * math.pi))
    return cen, rad


def neighbour_offsets(cen, rad, k=4):
    """Offsets of the k nearest other centres (ties to the lower index) / a_b,
    by brute force over all pairs; zeros where fewer than k others exist."""
    nb = cen.shape[0]
    out = np.zeros((nb, 3 * k))
    for b in range(nb):
        d2 = [(float(np.sum((cen[o] - cen[b]) ** 2)), o) for o in range(nb) if o != b]
        d2.sort()
        for j, (_, o) in enumerate(d2[:k]):
            out[b, 3 * j:3 * j + 3] = (cen[o] - cen[b]) / rad[b]
    return out


def features(xyz, s, phi, nb, nd, dirs, tri0, q=None):
    """Feature rows [nb, 174] and (if q is given) target rows [nb, 81]."""
    _, Gp = projector(dirs, tri0)
    cen, rad = bubble_frames(xyz, s, nb, nd)
    X = np.asarray(xyz, dtype=np.float64).reshape(nb, nd, 3)
    rho = np.linalg.norm(X - cen[:, None, :], axis=2) / rad[:, None]
    ph = np.asarray(phi, dtype=np.float64).reshape(nb, nd)
    feat = np.concatenate([rho @ Gp.T, ph @ Gp.T, neighbour_offsets(cen, rad)], axis=1)
    if q is None:
        return feat, None
    aq = np.asarray(q, dtype=np.float64).reshape(nb, nd) * rad[:, None]
    return feat, aq @ Gp.T


def synthesize(coef, xyz, s, nb, nd, dirs, tri0):
    """Guess q [nb * nd] from predicted coefficient rows coef [nb, 81]."""
    G, _ = projector(dirs, tri0)
    _, rad = bubble_frames(xyz, s, nb, nd)
    return ((np.asarray(coef, dtype=np.float64) @ G.T) / rad[:, None]).reshape(-1)


def bf16(x):
    """Round to bfloat16 (nearest, ties to even) via FP32; returns float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def standardise(x, mu, sd):
    return (np.asarray(x, dtype=np.float64) - mu) / sd
