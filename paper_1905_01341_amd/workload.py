"""Seeded synthetic inputs: icosphere bubble clusters and surface potentials.

This module builds inputs only. It holds none of the boundary-element
arithmetic (no areas, normals, kernels or sums), so the CPU oracle and the
GPU path can both consume what it produces without sharing any of the
method's code.

Mesh conventions (Section 3.1 and the tangential-velocity section of the
paper): a bubble surface is a closed triangulation whose vertices are the
collocation points; every triangle (r1, r2, r3) is ordered so that
(r2 - r1) x (r3 - r1) points out of the bubble into the liquid.

Workloads mirror the paper's clusters (Section 4: icosphere meshes with 642
vertices per bubble, clusters of up to thousands of bubbles):

* ``single``   one sphere R = 1, icosphere level 3, phi = 1/R + U[-0.1, 0.1]
* ``c100``     100 level-4 spheres, radii U[0.5, 1], centres in a cube of
               side 40, surface gap >= 0.5, phi ~ U[-1, 1]
* ``c1000``    1000 level-3 bubbles, radii U[0.5, 1], cube of side 90, gap
               >= 0.5 at bounding radius 1.05 R, shapes perturbed by real
               spherical harmonics of degree 2..8 (amplitude 0.05 R)
* ``c5000``    as ``c1000`` with 5000 bubbles in a cube of side 160
* ``torus1``   one toroidal bubble (genus 1, Section 3.7): major radius 1,
               tube radius 0.35, a 48 x 16 grid in the two angles (768
               vertices), phi = 1 + U[-0.1, 0.1]
* ``t100``     100 such tori, scales U[0.5, 1], random orientations, cube of
               side 30, bounding spheres >= 0.5 apart, phi ~ U[-1, 1]
* ``t1000``    1000 tori on a 42 x 14 grid (588 vertices each), cube of side
               90, phi per torus = U[-1, 1] + 0.1 x (random trigonometric
               polynomial of degree 1..3 in each angle, max-normalised)
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.special

SEED_BASE = 1905013410

# (name, seed offset) - seed = SEED_BASE + offset
WORKLOAD_SEEDS = {"single": 0, "c100": 1, "c1000": 2, "learned": 3, "c5000": 4, "torus1": 5, "t100": 6,
                  "t1000": 7}


@dataclasses.dataclass
class Cluster:
    """A bubble cluster: vertices, triangles and per-bubble ranges.

    xyz      float64 [nv, 3]   vertex positions (collocation points)
    tri      int32   [nt, 3]   vertex indices, outward orientation
    vtx_off  int64   [nb + 1]  bubble b owns vertices vtx_off[b]:vtx_off[b+1]
    tri_off  int64   [nb + 1]  bubble b owns triangles tri_off[b]:tri_off[b+1]
    centres  float64 [nb, 3]   bubble centres used for placement
    radii    float64 [nb]      unperturbed radii
    dirs     float64 [nv, 3]   unit direction of each vertex on its icosphere
                               (spherical bubbles; None for tori)
    angles   float64 [nv, 2]   (theta, phi) of each vertex on the unit torus:
                               theta around the tube, phi around the axis
                               (toroidal bubbles; None for spheres)
    """

    xyz: np.ndarray
    tri: np.ndarray
    vtx_off: np.ndarray
    tri_off: np.ndarray
    centres: np.ndarray
    radii: np.ndarray
    dirs: np.ndarray | None
    angles: np.ndarray | None = None

    @property
    def nv(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def nt(self) -> int:
        return int(self.tri.shape[0])

    @property
    def nb(self) -> int:
        return int(self.radii.shape[0])


_ICO_CACHE: dict[int, tuple[np.ndarray, np.ndarray]] = {}


def icosphere(level: int) -> tuple[np.ndarray, np.ndarray]:
    """Unit icosphere: 10*4^level + 2 vertices, 20*4^level triangles.

    Level 0 is the regular icosahedron; each level splits every triangle in
    four and pushes the new edge midpoints onto the unit sphere. Triangles
    are counter-clockwise seen from outside.
    """
    if level in _ICO_CACHE:
        v, f = _ICO_CACHE[level]
        return v.copy(), f.copy()
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    for _ in range(level):
        cache: dict[tuple[int, int], int] = {}

        def mid(a: int, b: int) -> int:
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    vv = np.array(verts, dtype=np.float64)
    ff = np.array(faces, dtype=np.int32)
    # orient outward: the icosahedron table above is CCW from outside, and
    # subdivision preserves orientation; assert it once.
    c = np.cross(vv[ff[:, 1]] - vv[ff[:, 0]], vv[ff[:, 2]] - vv[ff[:, 0]])
    assert np.all(np.einsum("ij,ij->i", c, vv[ff].mean(axis=1)) > 0)
    _ICO_CACHE[level] = (vv, ff)
    return vv.copy(), ff.copy()


def real_sh(nmax: int, dirs: np.ndarray, nmin: int = 0) -> np.ndarray:
    """Real orthonormal spherical harmonics of degrees nmin..nmax at unit
    directions ``dirs`` [k, 3]. Returns [k, (nmax+1)^2 - nmin^2], ordered by
    degree n, then order m = -n..n."""
    x, y, z = dirs[:, 0], dirs[:, 1], dirs[:, 2]
    theta = np.arccos(np.clip(z, -1.0, 1.0))
    az = np.arctan2(y, x)
    cols = []
    for n in range(nmin, nmax + 1):
        for m in range(-n, n + 1):
            yc = scipy.special.sph_harm_y(n, abs(m), theta, az)
            if m < 0:
                cols.append(np.sqrt(2.0) * (-1) ** m * yc.imag)
            elif m == 0:
                cols.append(yc.real)
            else:
                cols.append(np.sqrt(2.0) * (-1) ** m * yc.real)
    return np.stack(cols, axis=1)


def _place(rng: np.random.Generator, nb: int, side: float, rmin: float,
           rmax: float, gap: float, bound_factor: float):
    """Rejection-sample nb bubbles: centres U[0, side]^3, radii U[rmin, rmax],
    bounding spheres (bound_factor * R) at least ``gap`` apart."""
    centres = np.zeros((nb, 3))
    radii = np.zeros(nb)
    cell = 2.0 * rmax * bound_factor + gap
    grid: dict[tuple[int, int, int], list[int]] = {}
    k = 0
    tries = 0
    while k < nb:
        tries += 1
        if tries > 10000 * nb:
            raise RuntimeError("placement failed: cube too small for the gap rule")
        c = rng.uniform(0.0, side, size=3)
        r = rng.uniform(rmin, rmax)
        g = tuple(int(v) for v in np.floor(c / cell))
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for o in grid.get((g[0] + dx, g[1] + dy, g[2] + dz), ()):
                        d = np.linalg.norm(c - centres[o])
                        if d - bound_factor * (r + radii[o]) < gap:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            centres[k] = c
            radii[k] = r
            grid.setdefault(g, []).append(k)
            k += 1
    return centres, radii


def cluster(nb: int, level: int, side: float, rmin: float, rmax: float,
            gap: float, seed: int, perturb: float = 0.0,
            perturb_degrees: tuple[int, int] = (2, 8)) -> Cluster:
    """Build a cluster of nb icosphere bubbles (see module docstring)."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    v0, f0 = icosphere(level)
    nd = v0.shape[0]
    bound = 1.0 + perturb
    if nb == 1:
        centres = np.zeros((1, 3))
        radii = np.array([rmax])
    else:
        centres, radii = _place(rng, nb, side, rmin, rmax, gap, bound)
    xyz = np.empty((nb * nd, 3))
    if perturb > 0.0:
        ylm = real_sh(perturb_degrees[1], v0, nmin=perturb_degrees[0])
    for b in range(nb):
        rad = np.full(nd, radii[b])
        if perturb > 0.0:
            g = rng.standard_normal(ylm.shape[1])
            fvals = ylm @ g
            fvals /= np.max(np.abs(fvals))
            rad = radii[b] * (1.0 + perturb * fvals)
        xyz[b * nd:(b + 1) * nd] = centres[b] + rad[:, None] * v0
    tri = (f0[None, :, :] + (np.arange(nb, dtype=np.int64) * nd)[:, None, None])
    tri = tri.reshape(-1, 3).astype(np.int32)
    vtx_off = np.arange(nb + 1, dtype=np.int64) * nd
    tri_off = np.arange(nb + 1, dtype=np.int64) * f0.shape[0]
    dirs = np.tile(v0, (nb, 1))
    return Cluster(xyz, tri, vtx_off, tri_off, centres, radii, dirs)


TORUS_TUBE = 0.35  # tube radius of the template torus (major radius 1)


def torus(n_phi: int, n_theta: int, tube: float = TORUS_TUBE):
    """Torus of major radius 1 and tube radius ``tube`` on an n_phi x n_theta
    grid of the angles: vertex (i, k) at phi = 2 pi i / n_phi (around the
    axis z), theta = 2 pi k / n_theta (around the tube), position
    ((1 + tube cos theta) cos phi, (1 + tube cos theta) sin phi,
    tube sin theta), index i * n_theta + k. Each grid cell is split along
    its (i, k)-(i+1, k+1) diagonal; triangles are counter-clockwise seen
    from outside the tube. Returns (xyz, tri, angles [(theta, phi)])."""
    i, k = np.meshgrid(np.arange(n_phi), np.arange(n_theta), indexing="ij")
    ph = 2.0 * np.pi * i.ravel() / n_phi
    th = 2.0 * np.pi * k.ravel() / n_theta
    rho = 1.0 + tube * np.cos(th)
    xyz = np.stack([rho * np.cos(ph), rho * np.sin(ph), tube * np.sin(th)], axis=1)
    tri = []
    for a in range(n_phi):
        for b in range(n_theta):
            v00 = a * n_theta + b
            v10 = ((a + 1) % n_phi) * n_theta + b
            v01 = a * n_theta + (b + 1) % n_theta
            v11 = ((a + 1) % n_phi) * n_theta + (b + 1) % n_theta
            tri += [(v00, v10, v11), (v00, v11, v01)]
    tri = np.array(tri, dtype=np.int32)
    return xyz, tri, np.stack([th, ph], axis=1)


def _rotation(rng: np.random.Generator) -> np.ndarray:
    """A rotation matrix from a normalised Gaussian quaternion."""
    q = rng.standard_normal(4)
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def torus_cluster(nb: int, n_phi: int, n_theta: int, side: float, smin: float, smax: float,
                  gap: float, seed: int) -> Cluster:
    """nb toroidal bubbles: the template torus scaled by U[smin, smax],
    rotated at random and placed like ``cluster`` (bounding spheres of
    radius (1 + tube) x scale at least ``gap`` apart). ``radii`` holds the
    scales."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    v0, f0, a0 = torus(n_phi, n_theta)
    nd = v0.shape[0]
    if nb == 1:
        centres, scales = np.zeros((1, 3)), np.array([smax])
        rots = [np.eye(3)]
    else:
        centres, scales = _place(rng, nb, side, smin, smax, gap, 1.0 + TORUS_TUBE)
        rots = [_rotation(rng) for _ in range(nb)]
    xyz = np.empty((nb * nd, 3))
    for b in range(nb):
        xyz[b * nd:(b + 1) * nd] = centres[b] + scales[b] * (v0 @ rots[b].T)
    tri = (f0[None, :, :] + (np.arange(nb, dtype=np.int64) * nd)[:, None, None]).reshape(-1, 3).astype(np.int32)
    vtx_off = np.arange(nb + 1, dtype=np.int64) * nd
    tri_off = np.arange(nb + 1, dtype=np.int64) * f0.shape[0]
    return Cluster(xyz, tri, vtx_off, tri_off, centres, scales, None, np.tile(a0, (nb, 1)))


def make(name: str) -> tuple[Cluster, np.ndarray]:
    """Named workload -> (cluster, phi)."""
    seed = SEED_BASE + WORKLOAD_SEEDS[name]
    if name == "single":
        cl = cluster(1, 3, 0.0, 1.0, 1.0, 0.0, seed)
        rng = np.random.default_rng(np.random.PCG64(seed + 1000))
        phi = 1.0 / 1.0 + rng.uniform(-0.1, 0.1, size=cl.nv)
        return cl, phi
    if name == "c100":
        cl = cluster(100, 4, 40.0, 0.5, 1.0, 0.5, seed)
        rng = np.random.default_rng(np.random.PCG64(seed + 1000))
        return cl, rng.uniform(-1.0, 1.0, size=cl.nv)
    if name in ("c1000", "c5000"):
        nb, side = (1000, 90.0) if name == "c1000" else (5000, 160.0)
        cl = cluster(nb, 3, side, 0.5, 1.0, 0.5, seed, perturb=0.05)
        return cl, smooth_phi(cl, seed + 1000)
    if name == "torus1":
        cl = torus_cluster(1, 48, 16, 0.0, 1.0, 1.0, 0.0, seed)
        rng = np.random.default_rng(np.random.PCG64(seed + 1000))
        return cl, 1.0 + rng.uniform(-0.1, 0.1, size=cl.nv)
    if name == "t100":
        cl = torus_cluster(100, 48, 16, 30.0, 0.5, 1.0, 0.5, seed)
        rng = np.random.default_rng(np.random.PCG64(seed + 1000))
        return cl, rng.uniform(-1.0, 1.0, size=cl.nv)
    if name == "t1000":
        cl = torus_cluster(1000, 42, 14, 90.0, 0.5, 1.0, 0.5, seed)
        return cl, smooth_torus_phi(cl, seed + 1000)
    raise KeyError(name)


def smooth_torus_phi(cl: Cluster, seed: int, amp: float = 0.1, degree: int = 3) -> np.ndarray:
    """Per-torus potential: a uniform level U[-1, 1] plus a smooth variation
    (a random real trigonometric polynomial of degree 1..degree in each
    angle, max amplitude ``amp``)."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    nd = int(cl.vtx_off[1] - cl.vtx_off[0])
    th, ph = cl.angles[:nd, 0], cl.angles[:nd, 1]
    cols = []
    for n in range(degree + 1):
        for m in range(degree + 1):
            if n == 0 and m == 0:
                continue
            for fa in ((np.cos, np.sin) if n else (np.cos,)):
                for fb in ((np.cos, np.sin) if m else (np.cos,)):
                    cols.append(fa(n * th) * fb(m * ph))
    basis = np.stack(cols, axis=1)
    phi = np.empty(cl.nv)
    for b in range(cl.nb):
        f = basis @ rng.standard_normal(basis.shape[1])
        f /= np.max(np.abs(f))
        phi[cl.vtx_off[b]:cl.vtx_off[b + 1]] = rng.uniform(-1.0, 1.0) + amp * f
    return phi


def smooth_phi(cl: Cluster, seed: int, amp: float = 0.1) -> np.ndarray:
    """Per-bubble potential: a uniform level U[-1, 1] plus a smooth variation
    (real spherical harmonics of degree 1..4, max amplitude ``amp``)."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    nd = int(cl.vtx_off[1] - cl.vtx_off[0])
    ylm = real_sh(4, cl.dirs[:nd], nmin=1)
    phi = np.empty(cl.nv)
    for b in range(cl.nb):
        lev = rng.uniform(-1.0, 1.0)
        g = rng.standard_normal(ylm.shape[1])
        f = ylm @ g
        f /= np.max(np.abs(f))
        phi[cl.vtx_off[b]:cl.vtx_off[b + 1]] = lev + amp * f
    return phi


def rough_phi(cl: Cluster, seed: int) -> np.ndarray:
    """Per-vertex uniform U[-1, 1] potential (the roughest input)."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    return rng.uniform(-1.0, 1.0, size=cl.nv)


def subset_rows(n: int, k: int, seed: int) -> np.ndarray:
    """Seeded sorted choice of k distinct receiver indices out of n."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)
