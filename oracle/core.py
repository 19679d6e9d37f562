"""Oracle implementation: ctypes wrapper over bfm_oracle.c plus the solve.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bfm_oracle.c")
_LIB = os.path.join(_HERE, "libbfm_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle C source with gcc (FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        lib.bfmo_geometry.argtypes = [I64, P, I64, P, P, P, P]
        lib.bfmo_geometry.restype = ctypes.c_int
        lib.bfmo_sums.argtypes = [I64, P, P, P, P, I64, P, P, P, P, P, P]
        lib.bfmo_sums.restype = None
        lib.bfmo_offdiag_mvp.argtypes = [I64, P, P, P, D, P, D, P, I64, P, P]
        lib.bfmo_offdiag_mvp.restype = None
        lib.bfmo_dense.argtypes = [I64, P, P, P, P, P]
        lib.bfmo_dense.restype = None
        lib.bfmo_num_threads.argtypes = []
        lib.bfmo_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(_load().bfmo_num_threads())


def geometry(xyz, tri):
    """(s, n, area): vertex weights s_j, unit vertex normals n_j [nv, 3] and
    triangle areas A_k (ns1)."""
    lib = _load()
    xyz = _f64(xyz)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    nv, nt = xyz.shape[0], tri.shape[0]
    s = np.empty(nv)
    n = np.empty((nv, 3))
    area = np.empty(nt)
    rc = lib.bfmo_geometry(nv, _p(xyz), nt, _p(tri), _p(s), _p(n), _p(area))
    if rc != 0:
        raise ValueError(f"oracle geometry: invalid mesh (code {rc})")
    return s, n, area


def sums(xyz, s, n, phi=None, rows=None):
    """Direct sums over j != i (see bfmo_sums): dict of SM, VM, PM, VL, B."""
    lib = _load()
    xyz, s, n = _f64(xyz), _f64(s), _f64(n)
    nv = xyz.shape[0]
    rows = np.arange(nv, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nr = rows.shape[0]
    out = {k: np.empty(nr) for k in ("SM", "B")}
    for k in ("VM", "PM", "VL"):
        out[k] = np.empty((nr, 3))
    ph = None if phi is None else _f64(phi)
    lib.bfmo_sums(nv, _p(xyz), _p(s), _p(n), _p(ph), nr, _p(rows), _p(out["SM"]),
                  _p(out["VM"]), _p(out["PM"]), _p(out["VL"]), _p(out["B"]) if ph is not None else None)
    if ph is None:
        del out["B"]
    return out


def diagonals(xyz, s, n, rows=None, sm=None):
    """Singular diagonals (Section 3.3).

    M_ii = -1/2 - sum_{j!=i} M_ij                                      (s3)
    L_ii = n_i . [ sum_{j!=i} (M_ij r_j - L_ij n_j) + (1/2 + M_ii) r_i ]  (s5)

    Returns (M_ii, L_ii, L_ii_printed): L_ii is evaluated in the form
    n_i . [sum_{j!=i} M_ij (r_j - r_i) - sum_{j!=i} L_ij n_j], which equals
    s5 exactly because 1/2 + M_ii = -sum_{j!=i} M_ij; L_ii_printed is s5
    evaluated term by term as printed.
    """
    xyz, n = _f64(xyz), _f64(n)
    nv = xyz.shape[0]
    rows = np.arange(nv, dtype=np.int64) if rows is None else np.asarray(rows, dtype=np.int64)
    d = sums(xyz, s, n, None, rows) if sm is None else sm
    Mii = -0.5 - d["SM"]
    ni = n[rows]
    Lii = np.einsum("ij,ij->i", ni, d["VM"] - d["VL"])
    printed = d["PM"] - d["VL"] + (0.5 + Mii)[:, None] * xyz[rows]
    Lii_printed = np.einsum("ij,ij->i", ni, printed)
    return Mii, Lii, Lii_printed


def rhs(phi, B, rows=None):
    """b_i = -phi_i/2 + sum_j M_ij phi_j (eq3_1) with M_ii from s3, which is
    -phi_i + sum_{j!=i} M_ij (phi_j - phi_i)."""
    phi = _f64(phi)
    ph = phi if rows is None else phi[rows]
    return -ph + B


def offdiag_mvp(xyz, s, n, f=1.0, x=None, g=0.0, y=None, rows=None):
    """out_i = sum_{j!=i} (f L_ij x_j + g M_ij y_j) (eq3_27 without diagonal)."""
    lib = _load()
    xyz, s, n = _f64(xyz), _f64(s), _f64(n)
    nv = xyz.shape[0]
    rows = np.arange(nv, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty(rows.shape[0])
    xx = None if x is None else _f64(x)
    yy = None if y is None else _f64(y)
    if f != 0.0 and xx is None:
        raise ValueError("x required when f != 0")
    if g != 0.0 and yy is None:
        raise ValueError("y required when g != 0")
    lib.bfmo_offdiag_mvp(nv, _p(xyz), _p(s), _p(n), float(f), _p(xx), float(g), _p(yy),
                         rows.shape[0], _p(rows), _p(out))
    return out


def dense_offdiag(xyz, s, n):
    """Dense (L_off, M_off), zero diagonals (small meshes only)."""
    lib = _load()
    xyz, s, n = _f64(xyz), _f64(s), _f64(n)
    nv = xyz.shape[0]
    L = np.empty((nv, nv))
    M = np.empty((nv, nv))
    lib.bfmo_dense(nv, _p(xyz), _p(s), _p(n), _p(L), _p(M))
    return L, M


def system_dense(xyz, tri, phi):
    """Dense (L, M, b) of eq3_2 with both singular diagonals filled in."""
    s, n, _ = geometry(xyz, tri)
    L, M = dense_offdiag(xyz, s, n)
    Mii, Lii, _ = diagonals(xyz, s, n)
    L[np.diag_indices_from(L)] = Lii
    M[np.diag_indices_from(M)] = Mii
    b = -0.5 * _f64(phi) + M @ _f64(phi)
    return L, M, b


def matvec_L(xyz, s, n, Lii):
    """x -> L x with the full matrix (off-diagonal direct sum + L_ii x)."""
    def mv(x):
        return offdiag_mvp(xyz, s, n, 1.0, x) + Lii * x
    return mv


def gmres(matvec, b, x0=None, tol=1e-12, restart=50, maxit=2000, prec=None):
    """Restarted GMRES(m) (Saad and Schultz 1986), modified Gram-Schmidt
    Arnoldi, Givens rotations; stops when ||b - A x|| <= tol ||b|| (the true
    residual of the unpreconditioned system). prec, if given, is applied from
    the right (Arnoldi on A prec; x = x0 + prec(V y)), which changes the
    iterates but not the solution.

    Returns (x, info) with info = dict(iterations, restarts, rel_residual,
    converged)."""
    b = _f64(b)
    nrm_b = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
    if nrm_b == 0.0:
        return np.zeros_like(b), dict(iterations=0, restarts=0, rel_residual=0.0, converged=True)
    right = (lambda v: v) if prec is None else prec
    it = 0
    restarts = 0
    r = b - matvec(x)
    beta = np.linalg.norm(r)
    while True:
        if beta <= tol * nrm_b or it >= maxit:
            break
        m = restart
        V = np.zeros((m + 1, b.shape[0]))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        gvec = np.zeros(m + 1)
        gvec[0] = beta
        V[0] = r / beta
        k_used = 0
        for k in range(m):
            w = matvec(right(V[k]))
            it += 1
            for i in range(k + 1):
                H[i, k] = np.dot(V[i], w)
                w = w - H[i, k] * V[i]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] != 0.0:
                V[k + 1] = w / H[k + 1, k]
            for i in range(k):
                t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
                H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
                H[i, k] = t
            den = np.hypot(H[k, k], H[k + 1, k])
            cs[k] = H[k, k] / den
            sn[k] = H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            gvec[k + 1] = -sn[k] * gvec[k]
            gvec[k] = cs[k] * gvec[k]
            k_used = k + 1
            if abs(gvec[k + 1]) <= tol * nrm_b or it >= maxit:
                break
        y = np.zeros(k_used)
        for i in range(k_used - 1, -1, -1):
            y[i] = (gvec[i] - np.dot(H[i, i + 1:k_used], y[i + 1:k_used])) / H[i, i]
        x = x + right(V[:k_used].T @ y)
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        restarts += 1
    rel = beta / nrm_b
    return x, dict(iterations=it, restarts=restarts, rel_residual=rel, converged=rel <= tol)


def bubble_block_inverse(xyz, s, n, Lii, vtx_off):
    """Right preconditioner for GMRES: the exact inverse of every bubble's
    own diagonal block of L (dense LU per bubble, scipy). Bubble b owns
    vertices vtx_off[b]:vtx_off[b+1]."""
    import scipy.linalg as sla
    xyz, s, n = _f64(xyz), _f64(s), _f64(n)
    facs = []
    for b in range(len(vtx_off) - 1):
        o0, o1 = int(vtx_off[b]), int(vtx_off[b + 1])
        Lb, _ = dense_offdiag(xyz[o0:o1], s[o0:o1], n[o0:o1])
        Lb[np.diag_indices_from(Lb)] = Lii[o0:o1]
        facs.append((o0, o1, sla.lu_factor(Lb)))

    def apply(v):
        out = np.empty_like(v)
        for o0, o1, f in facs:
            out[o0:o1] = sla.lu_solve(f, v[o0:o1])
        return out
    return apply


def solve(xyz, tri, phi, method="gmres", tol=1e-12, restart=50, x0=None, maxit=2000, vtx_off=None,
          matvec_hook=None):
    """Solve L q = b (eq3_2) for q = dphi/dn at every vertex.

    method "gmres": restarted GMRES with direct-sum products (any N);
    method "gmres_bj": the same, right-preconditioned by the exact inverses
    of the bubbles' own diagonal blocks (vtx_off gives the bubble ranges);
    method "lu": dense LU of the assembled matrix (small N).
    matvec_hook(k) is called after every direct product (progress reports).
    Returns (q, info) with info carrying the diagonals and b.
    """
    xyz = _f64(xyz)
    phi = _f64(phi)
    s, n, _ = geometry(xyz, tri)
    d = sums(xyz, s, n, phi)
    Mii, Lii, Lii_p = diagonals(xyz, s, n, sm=d)
    b = rhs(phi, d["B"])
    info = dict(s=s, n=n, Mii=Mii, Lii=Lii, Lii_printed=Lii_p, b=b)
    if method == "lu":
        L, _ = dense_offdiag(xyz, s, n)
        L[np.diag_indices_from(L)] = Lii
        q = np.linalg.solve(L, b)
        nb = np.linalg.norm(b)
        info.update(iterations=0, rel_residual=np.linalg.norm(L @ q - b) / nb if nb > 0 else 0.0)
        return q, info
    base = matvec_L(xyz, s, n, Lii)
    count = [0]

    def mv(v):
        y = base(v)
        count[0] += 1
        if matvec_hook:
            matvec_hook(count[0])
        return y
    prec = None
    if method == "gmres_bj":
        if vtx_off is None:
            vtx_off = np.array([0, xyz.shape[0]])
        prec = bubble_block_inverse(xyz, s, n, Lii, vtx_off)
    elif method != "gmres":
        raise ValueError(method)
    q, gi = gmres(mv, b, x0=x0, tol=tol, restart=restart, maxit=maxit, prec=prec)
    info.update(gi)
    return q, info
