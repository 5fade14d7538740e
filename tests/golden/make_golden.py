"""Writes the stored expected values used by the full-size GPU parity tests.

Calls only the CPU oracle (and the seeded input generators).  For the 64^3
workload (64 boxes of 16^3, lognormal theta, corners + edges + faces) it
stores, at 512 seeded sample dofs: M^{-1} b, the PCG iterate after K
iterations from x0 = P_I b, and the converged solution; plus their norms, the
oracle's iteration count at rtol 1e-8 and its Lanczos condition estimate.

Run: python tests/golden/make_golden.py   (about 3 minutes on 8 cores)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import bddc_oracle as O  # noqa: E402
from paper_2410_14786_amd import workloads as W  # noqa: E402


def main():
    t0 = time.time()
    w = W.cfg_3d_64()
    P = O.BDDC(w.dim, w.nel, w.cuts, w.theta, w.constraints)
    print(f"oracle setup {time.time() - t0:.1f} s", flush=True)
    sample = np.sort(np.random.default_rng(1234).choice(P.n, size=512, replace=False))
    z = P.apply(w.b)
    ref = O.bddc_pcg(P, w.b, w.rtol)
    K = ref.iters - 2
    refK = O.bddc_pcg(P, w.b, 1e-300, maxit=K)
    out = {
        "workload": w.name,
        "source": "oracle/bddc_oracle.py via tests/golden/make_golden.py",
        "n_free": int(P.n),
        "n_coarse": int(P.n_coarse),
        "sample": sample.tolist(),
        "apply_b": {"values": z[sample].tolist(), "norm": float(np.linalg.norm(z))},
        "pcg": {"rtol": w.rtol, "iters": int(ref.iters), "cond_est": float(ref.cond_est),
                "relres_true": float(ref.relres_true), "values": ref.x[sample].tolist(),
                "norm": float(np.linalg.norm(ref.x))},
        "pcg_K": {"K": int(K), "values": refK.x[sample].tolist(), "norm": float(np.linalg.norm(refK.x))},
    }
    with open(os.path.join(HERE, "3d_64_sampled.json"), "w") as f:
        json.dump(out, f)
    print(f"done in {time.time() - t0:.1f} s: iters {ref.iters}, cond {ref.cond_est:.4f}", flush=True)


if __name__ == "__main__":
    main()
