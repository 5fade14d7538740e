"""The allocation-free apply (bddc_apply_noalloc) through the C ABI.

It must give what bddc_apply gives (the same kernels in the same order: the
same bits, and within the FP64 parity tolerance 1e-10 in any case) on two
calls in a row on different problems, the second smaller, since every call
on a GPU shares one fixed device workspace that keeps the last call's
contents; a problem whose apply workspace exceeds the fixed size is refused
with an error before any work is queued.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2410_14786_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def bd():
    from paper_2410_14786_amd import bddc
    return bddc


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def check_same(S, r):
    lib = bd().load_library()
    z_ref = torch.empty_like(r)
    z_na = torch.full_like(r, float("nan"))
    assert lib.bddc_apply(S.ctx, ctypes.c_void_p(r.data_ptr()),
                          ctypes.c_void_p(z_ref.data_ptr())) == 0
    assert lib.bddc_apply_noalloc(S.ctx, ctypes.c_void_p(r.data_ptr()),
                                  ctypes.c_void_p(z_na.data_ptr())) == 0
    torch.cuda.synchronize()
    a, b = z_na.cpu().numpy(), z_ref.cpu().numpy()
    assert np.all(np.isfinite(a))
    assert np.abs(a - b).max() <= 1e-10 * np.abs(b).max()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("full_space", [False, True], ids=["interface", "full_space"])
def test_noalloc_apply_matches_apply_twice(full_space):
    big = W.make_workload("t", 3, (16, 16, 16), (2, 2, 2), theta="lognormal", seed=4)
    small = W.make_workload("t", 3, (12, 10, 14), cuts=[[0, 5, 12], [0, 4, 7, 10], [0, 3, 9, 14]],
                            theta="lognormal", seed=5)
    S1 = bd().solver_for(big, full_space=full_space)
    S2 = bd().solver_for(small, full_space=full_space)
    rng = np.random.default_rng(21)
    check_same(S1, dev(rng.standard_normal(S1.n_free)))
    check_same(S2, dev(rng.standard_normal(S2.n_free)))    # second call, smaller problem
    check_same(S1, dev(rng.standard_normal(S1.n_free)))    # and back
    S1.close()
    S2.close()


def test_noalloc_apply_refuses_oversized_problem():
    # 128^3 workload with FP64 local factors: 4 * n_vec * 8 bytes > 64 MiB
    w = W.cfg_3d_128_uneven()
    S = bd().solver_for(w)
    r = dev(w.b)
    z = torch.zeros_like(r)
    lib = bd().load_library()
    rc = lib.bddc_apply_noalloc(S.ctx, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(z.data_ptr()))
    assert rc == -1
    assert b"fixed" in lib.bddc_last_error()
    torch.cuda.synchronize()
    assert not z.any()
    S.close()
