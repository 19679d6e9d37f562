"""The 1000-bubble cluster (642,000 nodes) at full size, in the bench's
configurations, against the oracle's solution (tests/golden/c1000_q_oracle.npy:
float32 copy of the FP64 direct-sum solve at relative residual 6.5e-12,
written by tests/golden/make_c1000_oracle.py). The bound is the metric's,
relative L2 error <= 1e-6, for the plain FP64 form and the tuned form."""
import json
import os

import numpy as np
import pytest

from paper_1905_01341_amd import bfm
from paper_1905_01341_amd import workload as wl

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def golden():
    cl, phi = wl.make("c1000")
    q = np.load(os.path.join(HERE, "golden", "c1000_q_oracle.npy")).astype(np.float64)
    meta = json.load(open(os.path.join(HERE, "golden", "c1000_q_oracle.json")))
    assert meta["nv"] == cl.nv and meta["rel_residual"] < 1e-10
    return cl, phi, q


@pytest.mark.parametrize("form", ["plain", "tuned"])
def test_c1000_solution_within_1e6_of_oracle(golden, form):
    cl, phi, q_ref = golden
    kw = dict(p=16, gmres_tol=1e-8, gmres_maxit=1000)
    if form == "tuned":
        kw.update(precond=bfm.PRECOND_SH_COARSE, precond_degree=12)
    sv = bfm.Solver(**kw)
    sv.set_cluster(cl)
    if form == "tuned":
        sv.autotune(1e-7)
    q, info = sv.solve(phi)
    err = float(np.linalg.norm(q - q_ref) / np.linalg.norm(q_ref))
    print(f"{form}: {info['iterations']} iterations, error vs oracle {err:.3e}")
    assert info["converged"] and err <= 1e-6
