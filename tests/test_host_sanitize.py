"""The host stage of bddc_setup (plan.cpp) built with AddressSanitizer and
UndefinedBehaviorSanitizer (g++, no GPU code) and run on the partitions of the
workloads and of the parity cases; its sizes must match the oracle's
independent count (free dofs, subdomains, coarse dofs, sum of local sizes)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import bddc_oracle as O
from paper_2410_14786_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2410_14786_amd", "csrc")


@pytest.fixture(scope="module")
def plan_check(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    out = str(tmp_path_factory.mktemp("asan") / "plan_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", f"-I{os.path.join(ROOT, 'include')}",
           os.path.join(CSRC, "plan_check.cpp"), os.path.join(CSRC, "plan.cpp"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
    return out


def case_line(w):
    cuts = list(w.cuts) + [np.array([0, 1])] * (3 - w.dim)
    nel = list(w.nel) + [1] * (3 - w.dim)
    parts = [str(w.dim)] + [str(n) for n in nel] + [str(w.constraints)]
    for c in cuts:
        parts += [str(len(c))] + [str(int(v)) for v in c]
    return " ".join(parts)


CASES = [
    lambda: W.cfg_2d_64(),
    lambda: W.make_workload("t", 2, (20, 24), cuts=[[0, 7, 13, 20], [0, 9, 24]]),
    lambda: W.make_workload("t", 3, (12, 10, 14), cuts=[[0, 5, 12], [0, 4, 7, 10], [0, 3, 9, 14]]),
    lambda: W.make_workload("t", 3, (40, 40, 40), cuts=[[0, 8, 32, 40]] * 3),
    lambda: W.make_workload("t", 3, (8, 8, 8), (2, 2, 2), constraints=W.CORNERS),
    lambda: W.make_workload("t", 2, (8, 8), (2, 2), constraints=W.ALL_PRIMAL),
    lambda: W.make_workload("t", 3, (9, 10, 11), (1, 1, 1)),
]


def test_planner_under_sanitizers(plan_check):
    ws = [c() for c in CASES]
    lines = [case_line(w) for w in ws]
    # the 128^3 and 64^3 workloads' partitions (planning only)
    big = [W.cfg_3d_128_uneven(), W.cfg_3d_64()]
    lines += [case_line(w) for w in big]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([plan_check], input="\n".join(lines) + "\n", capture_output=True, text=True, timeout=600,
                       env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    rows = [list(map(int, ln.split())) for ln in r.stdout.strip().splitlines()]
    assert len(rows) == len(lines)
    for w, row in zip(ws, rows):
        status, n_free, n_sub, n_coarse, sum_ni, max_nci, n_tiles, n_tasks = row
        P = O.BDDC(w.dim, w.nel, w.cuts, np.ones(w.n_el), w.constraints, factor=False)
        assert status == 0
        assert (n_free, n_sub, n_coarse) == (P.n, len(P.subs), P.n_coarse)
        assert sum_ni == sum(len(s.R) for s in P.subs)
        assert max_nci == max(s.C.shape[0] for s in P.subs)
        assert 0 < n_tasks <= n_tiles
    for row in rows[len(ws):]:
        assert row[0] == 0
    assert rows[len(ws)][1:4] == [2048383, 512, 2863]


def test_planner_rejects_bad_cuts_under_sanitizers(plan_check):
    bad = ["3 8 8 8 7 3 0 9 8 2 0 8 2 0 8",      # cut beyond nel
           "3 8 8 8 7 3 0 1 8 2 0 8 2 0 8",      # box of one element
           "2 8 8 1 3 2 0 8 3 0 4 4 2 0 1"]      # repeated cut
    r = subprocess.run([plan_check], input="\n".join(bad) + "\n", capture_output=True, text=True, timeout=120,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1"))
    assert r.returncode == 0, r.stderr[-4000:]
    assert all(int(ln.split()[0]) != 0 for ln in r.stdout.strip().splitlines())
