"""The two solver configurations the benchmark compares, in one place so that
the benchmark and the tests that pin it to the oracle run the same options.

* plain: the paper's method as printed - unpreconditioned restarted GMRES
  from a zero guess (Section 3.8), FP64 fast multipole products, no graph,
  no autotuning. Its GMRES tolerance is the loosest that still brings the
  1000-bubble solution within 1e-6 of the oracle's.
* tuned: the same system and stopping test (true FP64 residual), reached by
  mixed-precision iterative refinement (Arnoldi products in split-BF16
  arithmetic at a lower order p_lo, FP64 residuals at p; Section 3.11 weighs
  single against double precision), M2L translations of distant offsets at
  reduced orders (the same accuracy as the nearest offsets at order p), a
  right preconditioner, graph-replayed products and the autotuner's choice of
  p, p_lo, octree depth and M2L launch shape.

Argument marshalling only: every step runs in the HIP library.
"""
from __future__ import annotations

from . import bfm

PLAIN = dict(p=16, p_diag=0, leaf_target=64, lmax=0, m2l_shape=-1, gmres_tol=1e-8, gmres_restart=30,
             gmres_maxit=1000, precond=bfm.PRECOND_NONE, precond_degree=12, use_graph=0)
TUNED = dict(p=16, p_diag=0, leaf_target=64, lmax=0, m2l_shape=-1, gmres_tol=1e-7, gmres_restart=30,
             gmres_maxit=1000, precond=bfm.PRECOND_SH_COARSE, precond_degree=12, use_graph=0,
             precision=bfm.PREC_BF16X3, p_lo=0, ir_tol=1e-4, m2l_orders=1)
# product accuracy the autotuner must keep (relative to the p = 20 product)
TUNE_TOL = 1e-7
AUTOTUNE = {"plain": False, "tuned": True}


def options(form: str, **overrides) -> dict:
    base = {"plain": PLAIN, "tuned": TUNED}[form]
    opts = dict(base)
    for k, v in overrides.items():
        if v is not None:
            opts[k] = v
    return opts


def make_solver(cl, form: str, autotune: bool | None = None, tune_tol: float = TUNE_TOL, device: int = 0,
                **overrides):
    """A Solver for cluster `cl` in `form` ("plain" or "tuned"); returns
    (solver, autotune result dict or None)."""
    sv = bfm.Solver(device=device, **options(form, **overrides))
    sv.set_cluster(cl)
    tune = None
    if AUTOTUNE[form] if autotune is None else autotune:
        tune = sv.autotune(tune_tol)
    return sv, tune
