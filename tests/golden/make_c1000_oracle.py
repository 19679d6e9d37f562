"""Write the oracle's solution of the 1000-bubble cluster (642,000 nodes).

Calls only the oracle (oracle/) and the seeded input generator. Output:
tests/golden/c1000_q_oracle.npy (float32 copy of the FP64 solution; the
float32 rounding adds at most 6e-8 to a relative L2 error) and a JSON side
file with the solve's residual, iteration count and a checksum of the inputs.

Run from the repository root:  python tests/golden/make_c1000_oracle.py
(about an hour on 8 cores: every GMRES step is a 4.1e11-pair direct sum; the
GMRES is right-preconditioned by the exact inverses of the bubbles' own
blocks, which leaves the solution and the true-residual stopping test
unchanged and cuts the iteration count from over a hundred to about ten).
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1905_01341_amd import workload as wl  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden")


def main():
    cl, phi = wl.make("c1000")
    h = hashlib.sha256(cl.xyz.tobytes() + cl.tri.tobytes() + phi.tobytes()).hexdigest()
    t0 = time.time()
    q, info = oracle.solve(cl.xyz, cl.tri, phi, method="gmres_bj", tol=1e-11, restart=50,
                           vtx_off=cl.vtx_off,
                           matvec_hook=lambda k: print(f"  direct product {k} at {time.time() - t0:.0f} s",
                                                       flush=True))
    print(f"solve done: iterations={info['iterations']} rel_residual={info['rel_residual']:.3e}", flush=True)
    np.save(os.path.join(OUT, "c1000_q_oracle.npy"), q.astype(np.float32))
    meta = dict(workload="c1000", nv=cl.nv, nt=cl.nt, input_sha256=h,
                iterations=info["iterations"], rel_residual=float(info["rel_residual"]),
                gmres_tol=1e-11, restart=50, preconditioner="per-bubble dense block inverse (right)",
                q_norm2=float(np.linalg.norm(q)),
                threads=oracle.num_threads(), seconds=time.time() - t0)
    with open(os.path.join(OUT, "c1000_q_oracle.json"), "w") as f:
        json.dump(meta, f, indent=1)


if __name__ == "__main__":
    main()
