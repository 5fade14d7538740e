"""Full-size GPU checks, in the launch configuration bench.py times.

* 64^3, 64 boxes (the benchmark workload): sampled parity with stored oracle
  values (tests/golden/3d_64_sampled.json, written by make_golden.py from the
  oracle only): M^{-1} b, the iterate after K PCG steps and the iteration count.
* 128^3, 512 uneven boxes with inclusions (the headline workload): sampled
  parity with stored oracle values (tests/golden/3d_128_uneven_sampled.json,
  written by make_golden_128.py from the oracle only, 6 dofs of every box):
  M^{-1} b and the iterate after K PCG steps, element by element, in both
  iteration forms; the iteration count and Lanczos estimate; and, for the
  FP32-local forms (interface variant and FP32 local factors on the whole
  space), the true relative residual recomputed on the CPU from an
  independently assembled A and the error against the oracle's solution.
* 96^3, 216 boxes, adjoint gradient: the Euler identity (exact at any size) and
  central finite differences on 16 seeded elements.
"""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bddc_oracle as O
from paper_2410_14786_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def bd():
    from paper_2410_14786_amd import bddc
    return bddc


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def golden64():
    return json.load(open(os.path.join(GOLDEN, "3d_64_sampled.json")))


@pytest.fixture(scope="module")
def golden128():
    return json.load(open(os.path.join(GOLDEN, "3d_128_uneven_sampled.json")))


def sampled_close(v, g, key, tol):
    """Sampled entries of v against the stored oracle values: norm-wise over the
    sample, entry-wise against the oracle vector's largest magnitude, and the
    full vector's norm."""
    smp_vals = np.array(g[key]["values"])
    vs = v[np.array(g["sample"])]
    en = np.linalg.norm(vs - smp_vals) / np.linalg.norm(smp_vals)
    ee = np.abs(vs - smp_vals).max() / g[key]["maxabs"] if "maxabs" in g[key] else \
        np.abs(vs - smp_vals).max() / np.abs(smp_vals).max()
    enorm = abs(np.linalg.norm(v) - g[key]["norm"]) / g[key]["norm"]
    assert en <= tol and ee <= tol and enorm <= tol, (key, en, ee, enorm)
    return en, ee, enorm


def test_3d_64_sampled_parity_fp64(golden64):
    g = golden64
    w = W.cfg_3d_64()
    S = bd().solver_for(w)
    z = host(S.apply(dev(w.b)))
    say("3d_64 apply sampled rel err / entry-wise / norm", *sampled_close(z, g, "apply_b", 1e-10))
    K = g["pcg_K"]["K"]
    xK, info = S.solve(dev(w.b), 1e-15, maxit=K, raise_on_noconv=False)
    assert info["iters"] == K
    say("3d_64 PCG iterate K", K, "sampled rel err / entry-wise / norm",
        *sampled_close(host(xK), g, "pcg_K", 1e-10))
    x, info = S.solve(dev(w.b), w.rtol)
    say("3d_64 iters", info["iters"], "oracle", g["pcg"]["iters"], "relres", info["relres_true"],
        "cond", info["cond_est"], g["pcg"]["cond_est"])
    assert abs(info["iters"] - g["pcg"]["iters"]) <= 1
    assert info["relres_true"] <= w.rtol
    assert abs(info["cond_est"] - g["pcg"]["cond_est"]) <= 1e-4 * g["pcg"]["cond_est"]
    S.close()


def test_3d_64_fp32_local(golden64):
    g = golden64
    w = W.cfg_3d_64()
    S = bd().solver_for(w, local_bits=32)
    x, info = S.solve(dev(w.b), w.rtol)
    smp = np.array(g["sample"])
    xs = np.array(g["pcg"]["values"])
    e = np.linalg.norm(host(x)[smp] - xs) / np.linalg.norm(xs)
    say("3d_64 fp32-local iters", info["iters"], "relres_true", info["relres_true"], "sampled err vs oracle", e)
    assert info["relres_true"] <= w.rtol
    assert e <= 1e-6
    S.close()


def true_relres_cpu(w, x):
    A = O.assemble(O.Mesh(w.dim, w.nel), w.theta)
    return np.linalg.norm(w.b - A @ x) / np.linalg.norm(w.b)


@pytest.mark.parametrize("full_space", [False, True], ids=["interface", "full_space"])
def test_3d_128_sampled_parity_fp64(golden128, full_space):
    """The 128^3 workload (boxes of 8-24 elements per side) against the oracle:
    M^{-1} b and the K-step iterate on 6 sampled dofs of every box, element by
    element to 1e-10, the iteration count (+-1) and the Lanczos estimate."""
    g = golden128
    w = W.cfg_3d_128_uneven()
    S = bd().solver_for(w, full_space=full_space)
    say("3d_128 device GB", S.dev_bytes / 1e9, "full space", full_space)
    z = host(S.apply(dev(w.b)))
    say("3d_128 apply sampled rel err / entry-wise / norm", *sampled_close(z, g, "apply_b", 1e-10))
    K = g["pcg_K"]["K"]
    xK, info = S.solve(dev(w.b), 1e-15, maxit=K, raise_on_noconv=False)
    assert info["iters"] == K
    say("3d_128 PCG iterate K", K, "sampled rel err / entry-wise / norm",
        *sampled_close(host(xK), g, "pcg_K", 1e-10))
    x, info = S.solve(dev(w.b), w.rtol, maxit=1000)
    rr = true_relres_cpu(w, host(x))
    say("3d_128 fp64 iters", info["iters"], "oracle", g["pcg"]["iters"], "relres_true gpu", info["relres_true"],
        "cpu", rr, "cond", info["cond_est"], g["pcg"]["cond_est"], "solve ms", info["t_solve_ms"])
    assert abs(info["iters"] - g["pcg"]["iters"]) <= 1
    assert rr <= w.rtol * 1.01
    assert abs(info["cond_est"] - g["pcg"]["cond_est"]) <= 1e-6 * g["pcg"]["cond_est"]
    S.close()


@pytest.mark.parametrize("full_space", [False, True], ids=["interface_fp32_pc", "full_space_fp32_factors"])
def test_3d_128_fp32_local(golden128, full_space):
    """FP32 local solves on the 128^3 workload: full_space=True is the form with
    FP32 local Cholesky factors and FP32 triangular solves (FP64 CG, r1 and
    coarse problem); the interface variant keeps FP64 factors and applies the
    preconditioner's local solves in FP32.  No exact counterpart exists (parity
    unpinned): the true residual recomputed on the CPU must reach 1e-8, and the
    error against the oracle's converged solution on the sampled dofs is
    reported and bounded by 1e-5 (both solutions carry a 1e-8 residual)."""
    g = golden128
    w = W.cfg_3d_128_uneven(local_bits=32)
    S = bd().solver_for(w, full_space=full_space)
    x, info = S.solve(dev(w.b), w.rtol, maxit=1000)
    xh = host(x)
    rr = true_relres_cpu(w, xh)
    xs = np.array(g["pcg"]["values"])
    e = np.linalg.norm(xh[np.array(g["sample"])] - xs) / np.linalg.norm(xs)
    say("3d_128 fp32-local full_space", full_space, "iters", info["iters"], "oracle", g["pcg"]["iters"],
        "relres_true gpu", info["relres_true"], "cpu", rr, "sampled err vs oracle", e,
        "solve ms", info["t_solve_ms"])
    assert rr <= w.rtol * 1.01
    assert e <= 1e-5
    S.close()


@pytest.mark.timeout(600)
def test_3d_96_adjoint_gradient():
    w = W.cfg_3d_96_adjoint()
    bddc = bd()
    # observed field from the perturbed conductivity (FP64 local, tight tolerance)
    Sobs = bddc.Solver(w.dim, w.nel, w.cuts, w.theta_obs, w.constraints, local_bits=64)
    u_obs, _ = Sobs.solve(dev(w.b), 1e-12)
    Sobs.close()
    th = dev(w.theta).requires_grad_(True)
    b = dev(w.b)
    u = bddc.bddc_solve(th, b, 3, w.nel, w.cuts, w.constraints, rtol=1e-10, local_bits=32)
    res = u - u_obs
    loss = 0.5 * torch.sum(res * res)
    loss.backward()
    g = host(th.grad)
    u_h, uo_h = host(u.detach()), host(u_obs)
    # Euler identity: A is linear in theta, so u(c theta) = u / c and
    # sum_e theta_e dJ/dtheta_e = -(u - u_obs) . u
    lhs = float(w.theta @ g)
    rhs = -float((u_h - uo_h) @ u_h)
    say("euler identity", lhs, rhs)
    assert abs(lhs - rhs) <= 1e-6 * abs(rhs)
    # central differences, h = 1e-6, on 16 seeded elements, without cancellation:
    # A(theta +- h e_k) delta = -+ h K_k u, solved by delta <- -+h A^{-1} K_k (u + delta)
    # (a contraction for small h), then J(+-) - J = delta . (u - u_obs) + 0.5 |delta|^2
    S = bddc.Solver(w.dim, w.nel, w.cuts, w.theta, w.constraints, local_bits=64)
    uu, _ = S.solve(b, 1e-13)
    uu_h = host(uu)
    mesh = O.Mesh(3, w.nel)
    Kref = O.q1_reference_matrix(mesh.h)
    dofs_all = mesh.element_dofs(w.fd_elements)
    h = 1e-6
    worst = 0.0
    fd_vals = []
    for e, dofs in zip(w.fd_elements, dofs_all):
        m = dofs >= 0
        de = {}
        for sign in (+1, -1):
            delta = np.zeros_like(uu_h)
            for _ in range(3):
                v = uu_h[dofs[m]] + delta[dofs[m]]
                rhs_v = np.zeros_like(uu_h)
                rhs_v[dofs[m]] = -sign * h * (Kref[np.ix_(m, m)] @ v)
                dn, _ = S.solve(dev(rhs_v), 1e-13, maxit=2000)
                delta = host(dn)
            de[sign] = delta @ (uu_h - uo_h) + 0.5 * delta @ delta
        fd = (de[+1] - de[-1]) / (2 * h)
        fd_vals.append(fd)
        worst = max(worst, abs(fd - g[e]))
    scale = max(abs(v) for v in fd_vals)
    say("fd worst abs diff", worst, "scale", scale, "rel", worst / scale)
    assert worst <= 1e-6 * scale
    S.close()
