"""Writes the stored oracle values for the 128^3 uneven-box workload.

Calls only the CPU oracle (through its process-parallel driver, which runs the
oracle's own per-subdomain functions in worker processes) and the seeded input
generators.  Workload: 128^3 Q1 elements, 8^3 tensor boxes with lengths drawn
in [8, 24], one 1e-3 ellipsoid inclusion per box, corners + edge and face
averages, weights 1/kappa, rtol 1e-8 (Sec. 2, eqs. (1)-(5)).

Stored, at sample dofs (6 seeded dofs of every subdomain, interior and
interface alike, so that each box is checked): M^{-1} b, the PCG iterate after
K = iters - 2 steps from x0 = P_I b, and the converged solution; the norms and
largest magnitudes of those vectors; the oracle's iteration count at rtol 1e-8,
its Lanczos condition estimate and its true residual.

The local factors of 512 subdomains do not fit this host's memory at once, so
the factors are rebuilt at every application (keep_factors=False: the same
deterministic SuperLU factorisation each time, so the same operator).

Run: python tests/golden/make_golden_128.py [workers]   (about 30 minutes on 8 cores)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import parallel as OP  # noqa: E402
from paper_2410_14786_amd import workloads as W  # noqa: E402

PER_BOX = 6


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    t0 = time.time()
    w = W.cfg_3d_128_uneven()
    Q = OP.ParallelBDDC(w.dim, w.nel, w.cuts, w.theta, w.constraints, workers=workers, keep_factors=False)
    print(f"oracle setup {time.time() - t0:.1f} s ({Q.workers} workers), n {Q.n}, n_c {Q.n_coarse}", flush=True)
    rng = np.random.default_rng(4321)
    sample = np.unique(np.concatenate([rng.choice(s.R, size=PER_BOX, replace=False) for s in Q.P.subs]))
    t1 = time.time()
    z = Q.apply(w.b)
    print(f"apply {time.time() - t1:.1f} s", flush=True)
    iterates = {}

    def keep(k, x):
        iterates[k] = x.copy()
        print(f"  step {k} at {time.time() - t0:.0f} s", flush=True)

    ref = Q.pcg(w.b, w.rtol, callback=keep)
    K = ref.iters - 2
    xK = iterates[K]
    Q.close()

    def vec(v):
        return {"values": v[sample].tolist(), "norm": float(np.linalg.norm(v)), "maxabs": float(np.abs(v).max())}

    out = {
        "workload": w.name,
        "source": "oracle/bddc_oracle.py (per-subdomain steps run by oracle/parallel.py) via "
                  "tests/golden/make_golden_128.py",
        "n_free": int(Q.n),
        "n_coarse": int(Q.n_coarse),
        "sample": sample.tolist(),
        "apply_b": vec(z),
        "pcg": dict(rtol=w.rtol, iters=int(ref.iters), cond_est=float(ref.cond_est),
                    relres_true=float(ref.relres_true), **vec(ref.x)),
        "pcg_K": dict(K=int(K), **vec(xK)),
    }
    with open(os.path.join(HERE, "3d_128_uneven_sampled.json"), "w") as f:
        json.dump(out, f)
    print(f"done in {time.time() - t0:.1f} s: iters {ref.iters}, cond {ref.cond_est:.4f}, "
          f"relres_true {ref.relres_true:.3e}", flush=True)


if __name__ == "__main__":
    main()
