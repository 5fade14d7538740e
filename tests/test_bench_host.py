"""Host-side pieces of bench.py (no GPU): the element-to-dof map used by the
adjoint report's finite differences, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import bddc_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("nel", [(5, 4, 3), (2, 2, 2), (7, 3, 6)])
def test_element_free_dofs_match_oracle_mesh(nel):
    mesh = O.Mesh(3, nel)
    n_el = int(np.prod(nel))
    ref = mesh.element_dofs(np.arange(n_el))
    for e in range(n_el):
        want = sorted(int(d) for d in ref[e] if d >= 0)
        assert sorted(bench.element_free_dofs(nel, e)) == want


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_envelope_tile_count():
    """Tile counts of the triangular passes: a dense envelope (first column 0 in
    every tile row) gives the whole lower tile triangle; a band of half-width b
    tiles gives the band's tiles; the interior count covers ceil(n_I/64) rows."""
    T, TI = 5, 3
    n_R, n_I = 64 * T - 10, 64 * TI - 7
    dense = np.zeros(2 * T, dtype=np.int64)
    assert bench.envelope_tiles(dense, (n_R, n_I)) == (T * (T + 1) // 2, TI * (TI + 1) // 2, T)
    band = np.array([max(0, k - 1) for k in range(T)] * 2)
    rr, ii, t = bench.envelope_tiles(band, (n_R, n_I))
    assert rr == 1 + 2 * (T - 1) and ii == 1 + 2 * (TI - 1) and t == T


def test_envelope_bytes_never_exceed_dense_tiles():
    """Bytes counted from the envelope are at most those of the dense tile
    triangle (same vectors), and equal to them for a dense envelope."""
    from paper_2410_14786_amd import workloads as W
    w = W.make_workload("t", 3, (20, 18, 16), cuts=[[0, 9, 20], [0, 8, 18], [0, 16]], theta="one")
    sizes = bench.sub_sizes(w)
    dense_env, band_env = [], []
    for nR, nI, nci, nP in sizes:
        T = (nR + 63) // 64
        dense_env.append(bench.envelope_tiles(np.zeros(2 * T, dtype=np.int64), (nR, nI)))
        band_env.append(bench.envelope_tiles(np.array([max(0, k - 2) for k in range(T)] * 2), (nR, nI)))
    for lb in (4, 8):
        d = bench.algorithmic_bytes(w, lb, dense_env)
        b = bench.algorithmic_bytes(w, lb, band_env)
        for f in bench.FULL_FAMILIES:
            assert b[f] <= d[f]
        # the dense tile triangle holds at least the element triangle
        e = bench.algorithmic_bytes(w, lb)
        for f in bench.FULL_FAMILIES:
            assert d[f] >= e[f] - sum(nR * 64 * lb for nR, _, _, _ in sizes)


def test_traffic_records_are_consistent():
    """profiles/traffic.txt: every record's calibrated bytes follow from its two
    counter readings and factors, and bench.py finds a record only when it was
    taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    rows = [ln.split() for ln in open(path).read().splitlines() if ln and not ln.startswith("#")]
    assert rows
    keys = set()
    for key, sha, b, fk, wk, ff, wf in rows:
        assert key not in keys
        keys.add(key)
        assert len(sha) == 16 and all(c in "0123456789abcdef" for c in sha)
        assert abs(int(b) - (float(fk) * 1024 * float(ff) + float(wk) * 1024 * float(wf))) <= 2e-4 * int(b) + 1024
        assert 1.9 < float(ff) < 2.1 and 0.95 < float(wf) < 1.05
        workload, bits, kernel = key.split("/")
        got = bench.load_traffic(kernel, workload, int(bits))
        assert got == (int(b) if sha == bench.kernel_hash() else None)
