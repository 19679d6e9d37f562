"""Python binding of libbfm (ctypes, argument marshalling only).

Every numerical step runs in the HIP library; this module converts numpy
arrays or torch device tensors to pointers and back. It raises if the
compiled library is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbfm.so")

BFM_OK = 0
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENOCONV", -5: "EMESH", -6: "EUNSUPPORTED"}
PREC_FP64 = 0
PREC_FP32 = 1
PREC_BF16X3 = 2
PRECOND_NONE = 0
PRECOND_SH = 1
PRECOND_SH_COARSE = 2
GUESS_ZERO = 0
GUESS_GIVEN = 1
GUESS_LEARNED = 2
ABI_VERSION = 6
MLP_INPUTS = 174
MLP_OUTPUTS = 81
MLP_NUM_PARAMS = 656465
MLP_NORM_SIZE = 510


class BfmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bfm error {ERRORS.get(code, code)}: {msg}")
        self.code = code


class Physics(ctypes.Structure):
    _fields_ = [
        ("rho", ctypes.c_double),
        ("p0", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("kappa", ctypes.c_double),
        ("pa", ctypes.c_double),
        ("period", ctypes.c_double),
        ("forcing_sign", ctypes.c_double),
        ("g", ctypes.c_double * 3),
        ("alpha", ctypes.c_double),
        ("filter_degree", ctypes.c_int),
        ("guess", ctypes.c_int),
        ("collect", ctypes.c_int),
    ]


class TuneResult(ctypes.Structure):
    _fields_ = [
        ("p", ctypes.c_int),
        ("lmax", ctypes.c_int),
        ("m2l_shape", ctypes.c_int),
        ("candidates", ctypes.c_int),
        ("mvp_ms", ctypes.c_double),
        ("p_err", ctypes.c_double),
        ("p_lo", ctypes.c_int),
        ("p_diag", ctypes.c_int),
        ("diag_err", ctypes.c_double),
        ("p2p_shape", ctypes.c_int),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class StepInfo(ctypes.Structure):
    _fields_ = [
        ("scheme", ctypes.c_int),
        ("solves", ctypes.c_int),
        ("iterations", ctypes.c_int),
        ("t", ctypes.c_double),
        ("ms", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Options(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int),
        ("device", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("p", ctypes.c_int),
        ("p_diag", ctypes.c_int),
        ("lmax", ctypes.c_int),
        ("leaf_target", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("p_lo", ctypes.c_int),
        ("ir_tol", ctypes.c_double),
        ("gmres_tol", ctypes.c_double),
        ("gmres_restart", ctypes.c_int),
        ("gmres_maxit", ctypes.c_int),
        ("precond", ctypes.c_int),
        ("precond_degree", ctypes.c_int),
        ("use_graph", ctypes.c_int),
        ("m2l_shape", ctypes.c_int),
        ("m2l_orders", ctypes.c_int),
        ("p2p_shape", ctypes.c_int),
        ("near_corr", ctypes.c_int),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int),
        ("restarts", ctypes.c_int),
        ("matvecs", ctypes.c_int),
        ("converged", ctypes.c_int),
        ("rel_residual", ctypes.c_double),
        ("t_tree_ms", ctypes.c_double),
        ("t_diag_ms", ctypes.c_double),
        ("t_solve_ms", ctypes.c_double),
        ("t_guess_ms", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Load libbfm.so (raises FileNotFoundError if it was never built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} is missing: build it with paper_1905_01341_amd.build.build() "
            "(there is no fallback implementation)")
    # torch ships its own copy of the HIP runtime under the same soname. If
    # torch is installed, load it first so that libbfm binds to that copy:
    # one runtime per process, and device pointers of torch tensors are valid
    # in the library (a second runtime started later finds no GPU).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I = ctypes.c_int
    I64 = ctypes.c_int64
    D = ctypes.c_double
    sig = {
        "bfm_default_options": ([ctypes.POINTER(Options)], I),
        "bfm_create": ([ctypes.POINTER(Options), ctypes.POINTER(P)], I),
        "bfm_destroy": ([P], I),
        "bfm_set_options": ([P, ctypes.POINTER(Options)], I),
        "bfm_set_mesh": ([P, I64, P, I64, P, ctypes.c_int32, P, P], I),
        "bfm_set_positions": ([P, P], I),
        "bfm_set_sphere_template": ([P, ctypes.c_int32, P], I),
        "bfm_set_torus_template": ([P, ctypes.c_int32, P], I),
        "bfm_set_positions_dev": ([P, P], I),
        "bfm_geometry": ([P, P, P], I),
        "bfm_diagonals": ([P, P, P, P, P], I),
        "bfm_matvec": ([P, D, P, D, P, P, I, I, I], I),
        "bfm_solve": ([P, P, P, I, ctypes.POINTER(SolveInfo)], I),
        "bfm_solve_dev": ([P, P, P, I, ctypes.POINTER(SolveInfo)], I),
        "bfm_tree_stats": ([P, I, ctypes.POINTER(I64)], I),
        "bfm_last_error": ([], ctypes.c_char_p),
        "bfm_debug_operator": ([I, I, I, P, P], I),
        "bfm_debug_dgemm": ([I, I, I, I, P, P, P], I),
        "bfm_debug_spd_inverse": ([I, I, P, P], I),
        "bfm_debug_probe": ([I, I, I, P, P], I),
        "bfm_profile": ([P, I], I),
        "bfm_profile_read": ([P, I, P, P, P], I),
        "bfm_autotune": ([P, D, ctypes.POINTER(TuneResult)], I),
        "bfm_direct_dev": ([I64, P, P, P, D, P, D, P, I64, P, P, P], I),
        "bfm_direct_dev_noalloc": ([I64, P, P, P, D, P, D, P, I64, P, P, P], I),
        "bfm_default_physics": ([ctypes.POINTER(Physics)], I),
        "bfm_set_physics": ([P, ctypes.POINTER(Physics)], I),
        "bfm_state_set": ([P, P, P, D], I),
        "bfm_state_get": ([P, P, P, ctypes.POINTER(D)], I),
        "bfm_step": ([P, D, ctypes.POINTER(StepInfo)], I),
        "bfm_rhs": ([P, D, P, P, P, P, P, P], I),
        "bfm_mlp_init": ([P, ctypes.c_uint64], I),
        "bfm_mlp_set_params": ([P, P], I),
        "bfm_mlp_get_params": ([P, P], I),
        "bfm_mlp_set_norm": ([P, P], I),
        "bfm_mlp_get_norm": ([P, P], I),
        "bfm_mlp_forward": ([P, I64, P, P], I),
        "bfm_mlp_gradient": ([P, I64, P, P, P, ctypes.POINTER(D)], I),
        "bfm_mlp_adam_step": ([P, ctypes.c_float], I),
        "bfm_mlp_features": ([P, P, P, P, P], I),
        "bfm_mlp_collect_dev": ([P, P, P], I),
        "bfm_mlp_dataset": ([P, I, ctypes.POINTER(I64)], I),
        "bfm_mlp_fit": ([P, I, I, ctypes.c_float, ctypes.c_uint64, ctypes.POINTER(D)], I),
        "bfm_mlp_guess_dev": ([P, P, P], I),
        "bfm_mlp_guess": ([P, P, P], I),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(rc: int):
    if rc != BFM_OK:
        msg = load().bfm_last_error().decode(errors="replace")
        raise BfmError(rc, msg)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def default_options(**kw) -> Options:
    o = Options()
    _check(load().bfm_default_options(ctypes.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def debug_operator(p: int, kind: int, index: int):
    """Dense translation operator (see include/bfm_debug.h)."""
    P = p * p
    out = np.empty((P, P))
    d = np.zeros(3, dtype=np.int32)
    _check(load().bfm_debug_operator(p, kind, index, _ptr(out), _ptr(d)))
    return out, d


def debug_m2l_rotation(p: int, index: int):
    """Rotation-factored M2L operator `index` at order p (include/bfm_debug.h,
    kind 3): (A blocks per degree, T_z blocks per order, B blocks per
    degree), each a list of square arrays, and the offset d."""
    nr = p * (4 * p * p - 1) // 3
    nz = p * (p + 1) * (2 * p + 1) // 6
    out = np.empty(2 * nr + nz)
    d = np.zeros(3, dtype=np.int32)
    _check(load().bfm_debug_operator(p, 3, index, _ptr(out), _ptr(d)))

    def blocks(v, sizes):
        res, o = [], 0
        for s in sizes:
            res.append(v[o:o + s * s].reshape(s, s).copy())
            o += s * s
        return res
    rot = [2 * n + 1 for n in range(p)]
    return (blocks(out[:nr], rot), blocks(out[nr:nr + nz], [p - m for m in range(p)]),
            blocks(out[nr + nz:], rot), d)


PROBE_KINDS = {0: "fp64_mfma", 1: "fp64_fma", 2: "fp32_fma", 3: "fp64_pair", 4: "fp32_pair", 5: "bf16_mfma"}


def debug_probe(kind: int, iters: int, device: int = 0):
    """(ms, ops) of one ceiling-probe launch (include/bfm_debug.h)."""
    ms, ops = ctypes.c_double(), ctypes.c_double()
    _check(load().bfm_debug_probe(device, kind, iters, ctypes.byref(ms), ctypes.byref(ops)))
    return ms.value, ops.value


def debug_dgemm(A, B, device=0):
    """C = A B on the device with the library's FP64 MFMA GEMM (test hook)."""
    A = np.asfortranarray(A, dtype=np.float64)
    B = np.asfortranarray(B, dtype=np.float64)
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    C = np.empty((M, N), dtype=np.float64, order="F")
    _check(load().bfm_debug_dgemm(device, M, N, K, _ptr(A), _ptr(B), _ptr(C)))
    return C


def debug_spd_inverse(A, device=0):
    """The library's blocked Gauss-Jordan inverse of an SPD matrix (test hook)."""
    A = np.asfortranarray(A, dtype=np.float64)
    n = A.shape[0]
    out = np.empty((n, n), dtype=np.float64, order="F")
    _check(load().bfm_debug_spd_inverse(device, n, _ptr(A), _ptr(out)))
    return out


def _dptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def direct_dev(xyz_t, s_t, nrm_t, f=1.0, x_t=None, g=0.0, y_t=None, rows_t=None, out_t=None, nr=None,
               noalloc=False):
    """All-pairs off-diagonal product on torch device tensors (FP64, caller
    order; rows_t int64 or None); returns out_t. Runs on torch's current
    stream. noalloc: the allocation-free entry point (out_t must be given
    for a call that allocates nothing on the Python side either)."""
    import torch
    n = xyz_t.shape[0]
    if nr is None:
        nr = n if rows_t is None else rows_t.numel()
    if out_t is None:
        out_t = torch.empty(nr, dtype=torch.float64, device=xyz_t.device)
    st = torch.cuda.current_stream(xyz_t.device).cuda_stream
    fn = load().bfm_direct_dev_noalloc if noalloc else load().bfm_direct_dev
    _check(fn(n, _dptr(xyz_t), _dptr(s_t), _dptr(nrm_t), float(f), _dptr(x_t), float(g), _dptr(y_t), nr,
              _dptr(rows_t), _dptr(out_t), ctypes.c_void_p(st)))
    return out_t


class Solver:
    """One library handle (owns all device state for one mesh)."""

    def __init__(self, **opts):
        self.lib = load()
        self.opt = default_options(**opts)
        h = ctypes.c_void_p()
        _check(self.lib.bfm_create(ctypes.byref(self.opt), ctypes.byref(h)))
        self.h = h
        self.nv = 0
        self.nb = 0

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.bfm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_options(self, **kw):
        for k, v in kw.items():
            setattr(self.opt, k, v)
        _check(self.lib.bfm_set_options(self.h, ctypes.byref(self.opt)))

    def set_mesh(self, xyz, tri, vtx_off=None, tri_off=None):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        nb = 0
        vo = to = None
        if vtx_off is not None:
            vo = np.ascontiguousarray(vtx_off, dtype=np.int64)
            to = np.ascontiguousarray(tri_off, dtype=np.int64)
            nb = vo.shape[0] - 1
        _check(self.lib.bfm_set_mesh(self.h, xyz.shape[0], _ptr(xyz), tri.shape[0], _ptr(tri), nb,
                                     _ptr(vo), _ptr(to)))
        self.nv = xyz.shape[0]
        self.nb = max(nb, 1)

    def set_cluster(self, cl, template=True):
        self.set_mesh(cl.xyz, cl.tri, cl.vtx_off, cl.tri_off)
        nd = int(cl.vtx_off[1] - cl.vtx_off[0])
        if template and cl.nb * nd == cl.nv:
            if getattr(cl, "angles", None) is not None:
                self.set_torus_template(cl.angles[:nd])
            else:
                self.set_sphere_template(cl.dirs[:nd])

    def set_sphere_template(self, dirs):
        d = np.ascontiguousarray(dirs, dtype=np.float64)
        _check(self.lib.bfm_set_sphere_template(self.h, d.shape[0], _ptr(d)))

    def set_torus_template(self, angles):
        a = np.ascontiguousarray(angles, dtype=np.float64)
        _check(self.lib.bfm_set_torus_template(self.h, a.shape[0], _ptr(a)))

    def set_positions(self, xyz):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        _check(self.lib.bfm_set_positions(self.h, _ptr(xyz)))

    def geometry(self):
        s = np.empty(self.nv)
        n = np.empty((self.nv, 3))
        _check(self.lib.bfm_geometry(self.h, _ptr(s), _ptr(n)))
        return s, n

    def diagonals(self, phi):
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        Mii, Lii, b = (np.empty(self.nv) for _ in range(3))
        _check(self.lib.bfm_diagonals(self.h, _ptr(phi), _ptr(Mii), _ptr(Lii), _ptr(b)))
        return Mii, Lii, b

    def matvec(self, f=1.0, x=None, g=0.0, y=None, add_diag=False, precision=PREC_FP64, direct=False):
        xx = None if x is None else np.ascontiguousarray(x, dtype=np.float64)
        yy = None if y is None else np.ascontiguousarray(y, dtype=np.float64)
        out = np.empty(self.nv)
        _check(self.lib.bfm_matvec(self.h, float(f), _ptr(xx), float(g), _ptr(yy), _ptr(out),
                                   int(add_diag), int(precision), int(direct)))
        return out

    def solve(self, phi, q0=None, check=True, learned=False):
        """Host arrays in, (q, info dict) out. The initial guess is q0 if
        given, the trained network's prediction if learned, else zero."""
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        q = np.zeros(self.nv) if q0 is None else np.array(q0, dtype=np.float64)
        guess = GUESS_LEARNED if learned else (GUESS_GIVEN if q0 is not None else GUESS_ZERO)
        info = SolveInfo()
        rc = self.lib.bfm_solve(self.h, _ptr(phi), _ptr(q), guess, ctypes.byref(info))
        if check or rc not in (BFM_OK, -4):
            _check(rc)
        return q, info.as_dict()

    def solve_dev(self, phi_t, q_t, use_guess=False):
        """torch float64 device tensors (contiguous); q_t is overwritten.
        use_guess: False/True (zero or q_t as given) or one of GUESS_*."""
        import torch
        assert phi_t.dtype == torch.float64 and q_t.dtype == torch.float64
        assert phi_t.is_contiguous() and q_t.is_contiguous()
        assert phi_t.numel() == self.nv and q_t.numel() == self.nv
        torch.cuda.current_stream().synchronize()
        info = SolveInfo()
        _check(self.lib.bfm_solve_dev(self.h, ctypes.c_void_p(phi_t.data_ptr()),
                                      ctypes.c_void_p(q_t.data_ptr()), int(use_guess),
                                      ctypes.byref(info)))
        return info.as_dict()

    # kernel classes of bfm_profile_read (include/bfm.h)
    PRODUCT_KERNELS = ["p2p", "m2l", "m2m_l2l", "p2m", "l2p"]
    KERNEL_CLASSES = (PRODUCT_KERNELS + ["gmres", "tree", "diag"] + ["diag_" + k for k in PRODUCT_KERNELS]
                      + ["lo_" + k for k in PRODUCT_KERNELS])

    def profile(self, enable: bool):
        _check(self.lib.bfm_profile(self.h, int(enable)))

    def profile_read(self):
        k = len(self.KERNEL_CLASSES)
        ms = np.zeros(k)
        n = np.zeros(k, dtype=np.int64)
        fl = np.zeros(k)
        _check(self.lib.bfm_profile_read(self.h, k, _ptr(ms), _ptr(n), _ptr(fl)))
        return {k: dict(ms=float(ms[i]), launches=int(n[i]), flops=float(fl[i]))
                for i, k in enumerate(self.KERNEL_CLASSES)}

    def autotune(self, mvp_tol=1e-7):
        r = TuneResult()
        _check(self.lib.bfm_autotune(self.h, float(mvp_tol), ctypes.byref(r)))
        self.opt.p, self.opt.lmax, self.opt.m2l_shape = r.p, r.lmax, r.m2l_shape
        self.opt.p_diag = r.p_diag
        self.opt.p2p_shape = r.p2p_shape
        if r.p_lo:
            self.opt.p_lo = r.p_lo
        return r.as_dict()

    def tree_stats(self):
        keys = ["lmax", "leaves", "boxes", "near_pairs", "m2l_pairs", "tree_pairs", "max_leaf", "m2l_shape",
                "diag_m2l_shape"]
        st = (ctypes.c_int64 * len(keys))()
        _check(self.lib.bfm_tree_stats(self.h, len(keys), st))
        return {k: int(st[i]) for i, k in enumerate(keys)}

    # -- learned initial guess (include/bfm_mlp.h) ---------------------------

    def mlp_init(self, seed=0):
        _check(self.lib.bfm_mlp_init(self.h, int(seed)))

    def mlp_set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == MLP_NUM_PARAMS
        _check(self.lib.bfm_mlp_set_params(self.h, _ptr(p)))

    def mlp_get_params(self):
        p = np.empty(MLP_NUM_PARAMS, dtype=np.float32)
        _check(self.lib.bfm_mlp_get_params(self.h, _ptr(p)))
        return p

    def mlp_set_norm(self, norm):
        n = np.ascontiguousarray(norm, dtype=np.float32)
        assert n.size == MLP_NORM_SIZE
        _check(self.lib.bfm_mlp_set_norm(self.h, _ptr(n)))

    def mlp_get_norm(self):
        n = np.empty(MLP_NORM_SIZE, dtype=np.float32)
        _check(self.lib.bfm_mlp_get_norm(self.h, _ptr(n)))
        return n

    def mlp_forward(self, x):
        x = np.ascontiguousarray(x, dtype=np.float32)
        assert x.ndim == 2 and x.shape[1] == MLP_INPUTS
        y = np.empty((x.shape[0], MLP_OUTPUTS), dtype=np.float32)
        _check(self.lib.bfm_mlp_forward(self.h, x.shape[0], _ptr(x), _ptr(y)))
        return y

    def mlp_gradient(self, x, t):
        x = np.ascontiguousarray(x, dtype=np.float32)
        t = np.ascontiguousarray(t, dtype=np.float32)
        assert x.shape[0] == t.shape[0] and x.shape[1] == MLP_INPUTS and t.shape[1] == MLP_OUTPUTS
        g = np.empty(MLP_NUM_PARAMS, dtype=np.float32)
        loss = ctypes.c_double()
        _check(self.lib.bfm_mlp_gradient(self.h, x.shape[0], _ptr(x), _ptr(t), _ptr(g), ctypes.byref(loss)))
        return g, loss.value

    def mlp_adam_step(self, lr):
        _check(self.lib.bfm_mlp_adam_step(self.h, float(lr)))

    def mlp_features(self, phi, q=None):
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        qq = None if q is None else np.ascontiguousarray(q, dtype=np.float64)
        nb = self.nb
        feat = np.empty((nb, MLP_INPUTS), dtype=np.float32)
        targ = None if q is None else np.empty((nb, MLP_OUTPUTS), dtype=np.float32)
        _check(self.lib.bfm_mlp_features(self.h, _ptr(phi), _ptr(qq), _ptr(feat), _ptr(targ)))
        return feat, targ

    def mlp_collect_dev(self, phi_t, q_t):
        _check(self.lib.bfm_mlp_collect_dev(self.h, ctypes.c_void_p(phi_t.data_ptr()),
                                            ctypes.c_void_p(q_t.data_ptr())))

    def mlp_dataset(self, clear=False):
        n = ctypes.c_int64()
        _check(self.lib.bfm_mlp_dataset(self.h, int(clear), ctypes.byref(n)))
        return n.value

    def mlp_fit(self, epochs, batch=256, lr=1e-3, seed=0):
        loss = ctypes.c_double()
        _check(self.lib.bfm_mlp_fit(self.h, int(epochs), int(batch), float(lr), int(seed), ctypes.byref(loss)))
        return loss.value

    def mlp_guess(self, phi):
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        q = np.empty(self.nv)
        _check(self.lib.bfm_mlp_guess(self.h, _ptr(phi), _ptr(q)))
        return q

    def mlp_guess_dev(self, phi_t, q_t):
        _check(self.lib.bfm_mlp_guess_dev(self.h, ctypes.c_void_p(phi_t.data_ptr()),
                                          ctypes.c_void_p(q_t.data_ptr())))

    # -- time-step harness (include/bfm_step.h) ------------------------------

    def set_physics(self, **kw):
        ph = Physics()
        _check(self.lib.bfm_default_physics(ctypes.byref(ph)))
        for k, v in kw.items():
            if k == "g":
                for i in range(3):
                    ph.g[i] = float(v[i])
                continue
            if not hasattr(ph, k):
                raise KeyError(k)
            setattr(ph, k, v)
        _check(self.lib.bfm_set_physics(self.h, ctypes.byref(ph)))
        self.physics = ph

    def state_set(self, xyz, phi, t=0.0):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        _check(self.lib.bfm_state_set(self.h, _ptr(xyz), _ptr(phi), float(t)))

    def state_get(self):
        xyz = np.empty((self.nv, 3))
        phi = np.empty(self.nv)
        t = ctypes.c_double()
        _check(self.lib.bfm_state_get(self.h, _ptr(xyz), _ptr(phi), ctypes.byref(t)))
        return xyz, phi, t.value

    def step(self, dt):
        info = StepInfo()
        _check(self.lib.bfm_step(self.h, float(dt), ctypes.byref(info)))
        return info.as_dict()

    def rhs(self, t, xyz, phi):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        dx = np.empty((self.nv, 3))
        dp, q, H = (np.empty(self.nv) for _ in range(3))
        _check(self.lib.bfm_rhs(self.h, float(t), _ptr(xyz), _ptr(phi), _ptr(dx), _ptr(dp), _ptr(q), _ptr(H)))
        return dx, dp, q, H
