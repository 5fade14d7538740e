"""Process-parallel driver of the CPU oracle (test infrastructure only).

Only the test-suite, the scripts that write stored expected values and the
CPU-baseline leg of the benchmark may use it; the product path never does.

It runs the oracle's own per-subdomain functions (`setup_subdomain`,
`coarse_residual`, `coarse_interpolation`, `v2`, `interior_correction` of
oracle/bddc_oracle.py) in forked worker processes, each owning a fixed set of
subdomains, and adds their partial sums in the parent.  Nothing of the method
is rewritten here: the result is the oracle's M^{-1} r = v1 + v2 + v3 (Sec. 2,
eqs. (1)-(5)), up to the order in which the per-subdomain contributions are
summed (rounding only).

Two memory modes:
  * keep_factors=True: every worker keeps the sparse LU factors of its
    subdomains (fast applications; memory of all factors);
  * keep_factors=False: the factors are dropped after the coarse basis is
    formed and every application factors each KKT matrix (eq. (4)) and each
    interior block (eq. (5)) afresh, then drops it.  SuperLU is deterministic,
    so the operator is the same at every application; memory holds one
    subdomain's factor per worker.  This is how the 128^3 workload (512
    subdomains, tens of GB of factors) is run on a host with 64 GB.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import traceback
from typing import List, Optional, Sequence

import numpy as np

from oracle import bddc_oracle as O


def _limit_threads():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:  # pragma: no cover - threadpoolctl is installed here
        pass


def _worker(conn, P: "O.BDDC", idx: List[int], keep: bool):
    _limit_threads()
    subs = [P.subs[i] for i in idx]
    while True:
        msg = conn.recv()
        cmd, args = msg[0], msg[1:]
        try:
            if cmd == "stop":
                conn.send(("ok", None))
                break
            if cmd == "setup":
                out = []
                for i, s in zip(idx, subs):
                    O.setup_subdomain(s)
                    if not keep:
                        s.kkt_lu = None
                        s.Aii_lu = None
                    out.append((i, s.Ac))
                conn.send(("ok", out))
            elif cmd == "rc":
                conn.send(("ok", P.coarse_residual(args[0], subs)))
            elif cmd == "v12":
                r, uc = args
                v = P.coarse_interpolation(uc, subs) + P.v2(r, subs, refactor=not keep)
                conn.send(("ok", v))
            elif cmd == "v3":
                conn.send(("ok", P.interior_correction(args[0], subs, refactor=not keep)))
            else:
                conn.send(("error", f"unknown command {cmd}"))
        except Exception:
            conn.send(("error", traceback.format_exc()))


def _balance(costs: Sequence[float], nworkers: int) -> List[List[int]]:
    """Largest first onto the least loaded worker."""
    loads = [0.0] * nworkers
    parts: List[List[int]] = [[] for _ in range(nworkers)]
    for i in sorted(range(len(costs)), key=lambda k: -costs[k]):
        w = int(np.argmin(loads))
        parts[w].append(i)
        loads[w] += costs[i]
    return [sorted(p) for p in parts if p]


class ParallelBDDC:
    """The oracle's BDDC preconditioner with its subdomains spread over worker
    processes.  Attributes A, n, n_coarse, Ac, kappa mirror those of O.BDDC."""

    def __init__(self, dim: int, nel: Sequence[int], cuts: Sequence[np.ndarray], theta: np.ndarray,
                 constraints: int, workers: Optional[int] = None, keep_factors: bool = True,
                 weights: str = "kappa"):
        self.P = O.BDDC(dim, nel, cuts, theta, constraints, weights=weights, factor=False)
        nw = workers or os.cpu_count() or 1
        nw = max(1, min(nw, len(self.P.subs)))
        costs = [float(len(s.R)) ** 2 for s in self.P.subs]
        self.parts = _balance(costs, nw)
        ctx = mp.get_context("fork")
        self._conns, self._procs = [], []
        for idx in self.parts:
            a, b = ctx.Pipe()
            p = ctx.Process(target=_worker, args=(b, self.P, idx, keep_factors), daemon=True)
            p.start()
            self._conns.append(a)
            self._procs.append(p)
        self.workers = len(self._procs)
        for res in self._call_all(("setup",)):
            for i, Ac in res:
                self.P.subs[i].Ac = Ac
        self.P.assemble_coarse()

    # -- plumbing ---------------------------------------------------------------
    def _call_all(self, msg):
        for c in self._conns:
            c.send(msg)
        out = []
        for c in self._conns:
            status, val = c.recv()
            if status != "ok":
                raise RuntimeError(f"oracle worker failed:\n{val}")
            out.append(val)
        return out

    def close(self):
        for c in self._conns:
            try:
                c.send(("stop",))
                c.recv()
            except Exception:
                pass
        for p in self._procs:
            p.join(timeout=10)
        self._conns, self._procs = [], []

    def __del__(self):
        if getattr(self, "_procs", None):
            self.close()

    # -- the oracle's quantities ------------------------------------------------
    @property
    def A(self):
        return self.P.A

    @property
    def n(self):
        return self.P.n

    @property
    def n_coarse(self):
        return self.P.n_coarse

    @property
    def kappa(self):
        return self.P.kappa

    def apply(self, r: np.ndarray) -> np.ndarray:
        """M^{-1} r = v1 + v2 + v3 (Sec. 2): r_c, the coarse solve, v1 + v2 per
        worker, r1 = r - A (v1 + v2), v3 per worker."""
        r = np.asarray(r, dtype=np.float64)
        rc = np.zeros(self.n_coarse)
        for part in self._call_all(("rc", r)):
            rc += part
        uc = self.P.coarse_solve(rc)
        v12 = np.zeros(self.n)
        for part in self._call_all(("v12", r, uc)):
            v12 += part
        r1 = r - self.P.A @ v12
        return v12 + self.interior_correction(r1)

    def interior_correction(self, r1: np.ndarray) -> np.ndarray:
        v = np.zeros(self.n)
        for part in self._call_all(("v3", np.asarray(r1, dtype=np.float64))):
            v += part
        return v

    def pcg(self, b: np.ndarray, rtol: float, maxit: int = 1000, callback=None) -> "O.PCGResult":
        """BDDC-preconditioned CG from x0 = P_I b (O.bddc_pcg with this apply)."""
        x0 = self.interior_correction(b)
        return O.pcg(self.P.A, b, self.apply, rtol, maxit, x0=x0, callback=callback)
