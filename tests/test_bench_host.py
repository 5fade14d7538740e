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
