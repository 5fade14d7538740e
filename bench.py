"""Benchmark: BDDC-PCG solves/s on one MI355X.

Workload (default): 3D Q1 diffusion on a 128^3 element grid cut by seeded
random axis-aligned splits into 8^3 = 512 tensor boxes with edges of 8-24
elements (729-15625 dofs per box), one 1e-3 ellipsoid inclusion per box,
corner + edge + face constraints, uniform[-1,1] right-hand side, solved to
relative residual 1e-8.  A step is one warm BDDC-PCG solve (the preconditioner
is set up once beforehand, as when the matrix is reused across time steps);
inputs are resident in HBM when the timed region starts.

Prints one JSON line with the FP64 solve rate as `value` (CG restricted to the
interface dofs, the default of bddc_pcg_solve, kernels launched from the
host) and beside it: the FP32-local forms (FP32 local Cholesky factors and
triangular solves on the whole space, and the interface variant with the
preconditioner's local solves in FP32), the FP64 whole-space form (the
three-part preconditioner applied as written), graph replay, the setup
options (rho-scaling weights, coarse problem by CG), each with its iteration
count, true residual and error against stored oracle values; the roofline of
the dominant kernel (algorithmic bytes per launch over its HIP-event-timed
average duration); the 64^3 workload's rate as a secondary figure; the
adjoint-gradient check on the 96^3 workload; and a CPU-oracle baseline on a
bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FULL_FAMILIES = ["trsv_fwd_rr", "trsv_bwd_rr", "trsv_fwd_ii", "trsv_bwd_ii"]
GOLDEN = {"3d_128_uneven": "3d_128_uneven_sampled.json", "3d_64": "3d_64_sampled.json"}
TILE = 64 * 64
IFACE_FAMILIES = ["op", "pc"]
NB = 64


def sub_sizes(w):
    """Per-subdomain sizes of a tensor box partition: n_R (interior + non-corner
    interface rows of the local factor), n_I (interior rows), n_ci (constraints),
    n_P (corners)."""
    from paper_2410_14786_amd.workloads import CORNERS, EDGES, FACES
    dim = w.dim
    out = []
    nsub = [len(c) - 1 for c in w.cuts]
    for bidx in range(int(np.prod(nsub))):
        b, r = [], bidx
        for a in range(dim):
            b.append(r % nsub[a])
            r //= nsub[a]
        cnt, inner, ends = [], [], []
        for a in range(dim):
            lo, hi = int(w.cuts[a][b[a]]), int(w.cuts[a][b[a] + 1])
            n = w.nel[a]
            cnt.append(min(hi, n - 1) - max(lo, 1) + 1)
            inner.append(hi - lo - 1)
            ends.append(int(lo > 0) + int(hi < n))
        n_i = int(np.prod(cnt))
        n_I = int(np.prod(inner))
        corners = int(np.prod(ends)) if w.constraints & CORNERS else 0
        if dim == 3:
            edges = sum(ends[(c + 1) % 3] * ends[(c + 2) % 3] for c in range(3))
            faces = sum(ends)
        else:
            edges, faces = sum(ends), 0
        n_A = (edges if w.constraints & EDGES else 0) + (faces if w.constraints & FACES else 0)
        out.append((n_i - corners, n_I, n_A + corners, corners))
    return out


def envelope_tiles(env, sizes):
    """Tiles each pass of one subdomain streams: the lower tiles of L_RR inside
    the factor's envelope (tile (k, j) for fcol[k] <= j <= k, k < T) and of its
    interior block (fcol_ii[k] <= j <= k, k < TI); tiles left of the envelope are
    zero and neither stored into nor read."""
    n_R, n_I = sizes[0], sizes[1]
    T = (n_R + 63) // 64
    TI = (n_I + 63) // 64
    fc, fi = env[:T], env[T:2 * T]
    rr = int(sum(k - fc[k] + 1 for k in range(T)))
    ii = int(sum(k - fi[k] + 1 for k in range(TI)))
    return rr, ii, T


def algorithmic_bytes(w, local_bytes, env=None):
    """Bytes each kernel family must stream per launch.  Triangular passes: the
    tiles inside each factor's envelope (``env``: per subdomain the tile counts
    from envelope_tiles; without it the dense lower triangle), the border tile
    row (constraint rows) where it is read, and the vectors.  Interface form:
    the packed symmetric matrices and their FP64 input and output."""
    fam = {}
    s = sub_sizes(w)
    tri = lambda n: n * (n + 1) // 2
    tb = TILE * local_bytes
    if env is not None:
        rr_t = [e[0] for e in env]
        ii_t = [e[1] for e in env]
        border = [e[2] if nci else 0 for e, (nR, nI, nci, nP) in zip(env, s)]
        fam["trsv_fwd_rr"] = sum(rr * tb + bt * tb + nR * (8 + 8 + 4 + local_bytes)
                                 for rr, bt, (nR, nI, nci, nP) in zip(rr_t, border, s))
        fam["trsv_bwd_rr"] = sum(rr * tb + bt * tb + nR * (8 + 2 * local_bytes)
                                 for rr, bt, (nR, nI, nci, nP) in zip(rr_t, border, s))
        fam["trsv_fwd_ii"] = sum(ii * tb + nI * (8 + 4 + local_bytes) for ii, (nR, nI, nci, nP) in zip(ii_t, s))
        fam["trsv_bwd_ii"] = sum(ii * tb + nI * (8 + 8 + 4 + local_bytes) for ii, (nR, nI, nci, nP) in zip(ii_t, s))
    else:
        fam["trsv_fwd_rr"] = sum(tri(nR) * local_bytes + nci * nR * local_bytes + nR * (8 + 8 + 4 + local_bytes)
                                 for nR, nI, nci, nP in s)
        fam["trsv_bwd_rr"] = sum(tri(nR) * local_bytes + nci * nR * local_bytes + nR * (8 + 2 * local_bytes)
                                 for nR, nI, nci, nP in s)
        fam["trsv_fwd_ii"] = sum(tri(nI) * local_bytes + nI * (8 + 4 + local_bytes) for nR, nI, nci, nP in s)
        fam["trsv_bwd_ii"] = sum(tri(nI) * local_bytes + nI * (8 + 8 + 4 + local_bytes) for nR, nI, nci, nP in s)
    # interface form: the operator (always FP64) streams the lower triangle of
    # the local Schur complement on n_G + n_P rows (n_G = n_R - n_I interface
    # rows, n_P corners), the preconditioner (local precision) that of X^T X on
    # n_G rows plus the n_ci x n_G border block; each reads its FP64 input and
    # writes its FP64 output once
    fam["op"] = sum(tri(nR - nI + nP) * 8 + (nR - nI + nP) * (8 + 8) for nR, nI, nci, nP in s)
    fam["pc"] = sum(tri(nR - nI) * local_bytes + nci * (nR - nI) * local_bytes + (nR - nI) * (8 + 8) + nci * 8
                    for nR, nI, nci, nP in s)
    return fam


def kernel_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2410_14786_amd", "csrc", "kernels.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload, local_bits):
    """HBM traffic per launch measured by rocprofv3 counters, if the record in
    profiles/traffic.txt was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    key = f"{workload}/{local_bits}/{kernel}"
    for ln in lines:
        parts = ln.split()
        if ln.startswith("#") or len(parts) < 3 or parts[0] != key:
            continue
        return int(parts[2]) if parts[1] == kernel_hash() else None
    return None


def load_golden(workload):
    name = GOLDEN.get(workload)
    if name is None:
        return None
    path = os.path.join(ROOT, "tests", "golden", name)
    return json.load(open(path)) if os.path.exists(path) else None


def golden_error(x, golden):
    """Error of a solution against the oracle's converged solution on the
    stored sample dofs: norm-wise over the sample and entry-wise against the
    oracle vector's largest magnitude."""
    if golden is None:
        return None
    smp = np.array(golden["sample"])
    ref = np.array(golden["pcg"]["values"])
    d = x[smp] - ref
    mx = golden["pcg"].get("maxabs", float(np.abs(ref).max()))
    return {"sampled_rel": float(np.linalg.norm(d) / np.linalg.norm(ref)),
            "sampled_entrywise": float(np.abs(d).max() / mx), "oracle_iters": golden["pcg"]["iters"],
            "samples": int(len(smp))}


def run_gpu(w, steps, warmup, local_bits, use_graph=False, full_space=False, autotune=True, timing=True,
            rho_scaling=False, coarse_cg=False, golden=None):
    import torch
    from paper_2410_14786_amd import bddc
    families = FULL_FAMILIES if full_space else IFACE_FAMILIES + ["trsv_fwd_ii", "trsv_bwd_ii"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = bddc.solver_for(w, local_bits=local_bits, use_graph=use_graph, full_space=full_space,
                        rho_scaling=rho_scaling, coarse_cg=coarse_cg)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    tune = S.autotune(cache="") if autotune else None
    env = []
    for i in range(S.n_sub):
        sz = S.debug_read("sizes", i)
        env.append(envelope_tiles(S.debug_read("envelope", i).astype(np.int64), (int(sz[0]), int(sz[1]))))
    b = torch.as_tensor(w.b, dtype=torch.float64, device="cuda")
    x = torch.empty_like(b)
    info = None
    for _ in range(warmup):
        _, info = S.solve(b, w.rtol, out=x)
    S.set_timing(timing)
    for f in families + ["apply"]:
        S.kernel_time(f)   # reset counters
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    for _ in range(steps):
        _, info = S.solve(b, w.rtol, out=x)
        iters.append(info["iters"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    fam = {f: S.kernel_time(f) for f in families + ["apply"]}
    S.set_timing(False)
    flops, factor_ms = S.setup_stats()
    xh = x.cpu().numpy()
    res = {"setup_s": setup_s, "elapsed_s": elapsed, "iters": iters, "info": info, "kernels": fam,
           "dev_bytes": S.dev_bytes, "families": families, "tuning": tune, "factor_flops": flops,
           "factor_ms": factor_ms, "env": env, "full_space": full_space,
           "err_vs_oracle": golden_error(xh, golden)}
    S.close()
    del S
    torch.cuda.empty_cache()
    return res


def element_free_dofs(nel, e):
    """Free dofs of Q1 element e of the structured cube (elements and free nodes
    numbered x fastest; boundary nodes are not free)."""
    nx, ny, nz = nel
    ex, ey, ez = e % nx, (e // nx) % ny, e // (nx * ny)
    out = []
    for c in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                ix, iy, iz = ex + a, ey + b, ez + c
                if 1 <= ix <= nx - 1 and 1 <= iy <= ny - 1 and 1 <= iz <= nz - 1:
                    out.append((ix - 1) + (nx - 1) * ((iy - 1) + (ny - 1) * (iz - 1)))
    return out


def adjoint_report(n_fd=4, h=1e-6):
    """Gradient of J = |u - u_obs|^2 / 2 with respect to the element
    conductivities on the 96^3 adjoint workload (6^3 boxes of 16^3, FP32 local
    factors): the differentiable solve (setup, forward and adjoint BDDC-PCG, the
    element kernel) timed from the host; the Euler identity (A is linear in theta,
    so theta . dJ/dtheta = -(u - u_obs) . u); and central differences on n_fd
    seeded elements without cancellation: A(theta +- h e_k) u_+- = b is solved as
    the correction delta = -+ h A^{-1} K_k (u + delta) (a contraction for small h;
    K_k v is read off the element-gradient kernel with unit vectors), and
    J(+-) - J = delta . (u - u_obs) + |delta|^2 / 2."""
    import torch
    from paper_2410_14786_amd import bddc
    from paper_2410_14786_amd import workloads as W
    w = W.cfg_3d_96_adjoint(n_fd=n_fd)
    dev = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda")
    b = dev(w.b)
    S_obs = bddc.Solver(w.dim, w.nel, w.cuts, w.theta_obs, w.constraints, local_bits=64)
    u_obs, _ = S_obs.solve(b, 1e-12)
    S_obs.close()
    th = dev(w.theta).requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u = bddc.bddc_solve(th, b, 3, w.nel, w.cuts, w.constraints, rtol=1e-10, local_bits=32)
    loss = 0.5 * torch.sum((u - u_obs) ** 2)
    loss.backward()
    torch.cuda.synchronize()
    grad_s = time.perf_counter() - t0
    g = th.grad.detach().cpu().numpy()
    u_h, uo_h = u.detach().cpu().numpy(), u_obs.cpu().numpy()
    lhs, rhs = float(w.theta @ g), -float((u_h - uo_h) @ u_h)
    S = bddc.Solver(w.dim, w.nel, w.cuts, w.theta, w.constraints, local_bits=64)
    uu, _ = S.solve(b, 1e-13)
    uu_h = uu.cpu().numpy()
    unit = torch.zeros_like(b)
    worst, scale = 0.0, 0.0
    for e in w.fd_elements:
        dofs = element_free_dofs(w.nel, int(e))
        de = {}
        for sign in (+1, -1):
            delta = np.zeros_like(uu_h)
            for _ in range(3):
                v = dev(uu_h + delta)
                rhs_v = np.zeros_like(uu_h)
                for d in dofs:
                    unit[d] = 1.0
                    # elem_grad gives -unit_e^T K_e v_e, i.e. -(K_e v)_d
                    rhs_v[d] = sign * h * float(S.elem_grad(unit, v)[int(e)])
                    unit[d] = 0.0
                dn, _ = S.solve(dev(rhs_v), 1e-13, maxit=2000)
                delta = dn.cpu().numpy()
            de[sign] = delta @ (uu_h - uo_h) + 0.5 * delta @ delta
        fd = (de[+1] - de[-1]) / (2 * h)
        worst = max(worst, abs(fd - g[int(e)]))
        scale = max(scale, abs(fd))
    S.close()
    torch.cuda.empty_cache()
    return {"workload": w.name, "n_free": int(w.n_free), "local_bits": 32, "grad_s_with_setup": grad_s,
            "euler_rel": abs(lhs - rhs) / abs(rhs), "fd_elements": len(w.fd_elements), "fd_h": h,
            "fd_rel_worst": worst / scale if scale > 0 else None}


def cpu_baseline(w_full, full_iters, workers=None):
    """The oracle on a bounded sample of the workload, one worker process per
    host core (oracle/parallel.py runs the oracle's per-subdomain steps in
    forked workers, BLAS limited to one thread each).  128^3 workload: the
    4x4x4 block of boxes at the origin (64 of the 512 subdomains, the same cut
    positions and the same inclusion coefficients), as a problem of its own
    with a fresh uniform[-1,1] right-hand side; 64^3: 2x2x2 boxes of 16^3 with
    the same lognormal law.  The sample's solve time (setup excluded, as for
    the GPU rate) is scaled by the subdomain count and by the iteration ratio to
    give solves/s for the full workload."""
    import platform
    from oracle import parallel as OP
    from paper_2410_14786_amd import workloads as W
    nsub_full = int(np.prod(w_full.nsub))
    if w_full.name.startswith("3d_q1_128"):
        k = 4
        cuts = [np.asarray(c[:k + 1], dtype=np.int64) for c in w_full.cuts]
        nel = tuple(int(c[-1]) for c in cuts)
        full_nel = w_full.nel
        ex, ey, ez = np.meshgrid(np.arange(nel[0]), np.arange(nel[1]), np.arange(nel[2]), indexing="ij")
        eidx = (ex + full_nel[0] * (ey + full_nel[1] * ez)).transpose(2, 1, 0).ravel()
        theta = w_full.theta[eidx]
        rng = np.random.default_rng(99)
        b = rng.uniform(-1.0, 1.0, int(np.prod([n - 1 for n in nel])))
        what = (f"oracle BDDC-PCG on the 4x4x4 block of boxes at the origin of the 128^3 workload "
                f"({nel[0]}x{nel[1]}x{nel[2]} elements, 64 of the 512 subdomains, same cuts and inclusions)")
        dim, cons, rtol = 3, w_full.constraints, w_full.rtol
    else:
        ws = W.make_workload("sample", 3, (32, 32, 32), (2, 2, 2), theta="lognormal", rtol=1e-8, seed=0)
        cuts, nel, theta, b = ws.cuts, ws.nel, ws.theta, ws.b
        what = "oracle BDDC-PCG on 32^3 elements, 2x2x2 boxes of 16^3 (8 of the 64 subdomains)"
        dim, cons, rtol = 3, ws.constraints, ws.rtol
    nsub_s = int(np.prod([len(c) - 1 for c in cuts]))
    workers = workers or min(os.cpu_count() or 1, 16, nsub_s)
    t0 = time.perf_counter()
    Q = OP.ParallelBDDC(dim, nel, cuts, theta, cons, workers=workers, keep_factors=True)
    setup = time.perf_counter() - t0
    try:
        reps, total = 0, 0.0
        while reps < 20 and (reps == 0 or total < 10.0):
            t0 = time.perf_counter()
            res = Q.pcg(b, rtol)
            total += time.perf_counter() - t0
            reps += 1
    finally:
        Q.close()
    t = total / reps
    scale = (nsub_full / nsub_s) * (full_iters / max(res.iters, 1))
    cpu = platform.processor() or platform.machine()
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                cpu = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": 1.0 / (t * scale), "unit": "solves/s", "cores": Q.workers, "kind": "oracle",
            "cpu": cpu, "host_cpus": os.cpu_count(),
            "sample": f"{what}; {res.iters} iterations; {reps} solves in {total:.1f} s ({t:.2f} s each) with "
                      f"{Q.workers} worker processes (one per core, BLAS 1 thread each; oracle setup {setup:.1f} s "
                      f"not timed); scaled x{nsub_full / nsub_s:g} for subdomains and x{full_iters}/{res.iters} "
                      f"for iterations"}


def copy_bandwidth(torch):
    """HBM bandwidth of two plain streams on this GPU (GB/s), reference points
    beside the datasheet peak: PyTorch's device copy (bytes read plus bytes
    written) and its sum of a vector (bytes read).  They are not ceilings: a
    read stream written for the purpose (non-temporal 16-byte loads, whole
    tiles per workgroup) moves more."""
    n = (1 << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)

    def timed(fn):
        fn()
        ts = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3)
        return float(np.median(ts))

    copy = 2 * n * 8 / timed(lambda: dst.copy_(src)) / 1e9
    read = n * 8 / timed(lambda: src.sum()) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return copy, read


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="3d_128_uneven")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-full-space", action="store_true")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the run that replays captured HIP graphs")
    ap.add_argument("--local-bits", type=int, default=64)
    ap.add_argument("--no-rho", action="store_true", help="skip the run with coefficient-aware weights")
    ap.add_argument("--no-coarse-cg", action="store_true", help="skip the run with the coarse problem by CG")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the gradient check on the 96^3 adjoint workload")
    ap.add_argument("--no-secondary", action="store_true", help="skip the 64^3 workload's secondary rate")
    ap.add_argument("--only-main", action="store_true",
                    help="only the main runs (untimed and timed); for profiling")
    ap.add_argument("--main-form", choices=["interface", "full"], default="interface",
                    help="iteration form of the main runs (full: CG on the whole space)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 512 MiB device copy first (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the whole problem lives on one MI355X); --gpus {args.gpus} "
              f"is not supported", file=sys.stderr)
        sys.exit(2)
    if args.only_main:
        args.no_cpu_baseline = args.no_fp32 = args.no_full_space = args.no_graph = True
        args.no_rho = args.no_coarse_cg = args.no_adjoint = args.no_secondary = True
    import torch
    from paper_2410_14786_amd import workloads as W
    if args.copy_calibration:
        n = 512 * 1024 * 1024 // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # (not in counter runs, whose calibration copy must be the only large copy)
    copy_gbs, read_gbs = (None, None) if args.copy_calibration else copy_bandwidth(torch)
    w = W.WORKLOADS[args.workload]()
    golden = load_golden(args.workload)
    print(f"[bench] workload {w.name}: n_free {w.n_free}, {int(np.prod(w.nsub))} subdomains", file=sys.stderr,
          flush=True)
    main_bits = args.local_bits
    runs = {}

    def run(name, *a, **k):
        print(f"[bench] run {name}", file=sys.stderr, flush=True)
        runs[name] = run_gpu(w, args.steps, args.warmup, *a, golden=golden, **k)
        r = runs[name]
        print(f"[bench] {name}: {1000 * r['elapsed_s'] / args.steps:.2f} ms/solve, iters {r['iters'][-1]}, "
              f"setup {r['setup_s']:.2f} s", file=sys.stderr, flush=True)

    # `value`: kernels launched from the host with no timing events (the host
    # stays ahead of the GPU, and eager launches read their arguments from device
    # memory, which graph kernel nodes on this ROCm do not); the same solves with
    # dispatch-recorded events give the per-kernel times and the roofline; the
    # graph-replay rate is reported beside them
    main_full = args.main_form == "full"
    run("main", main_bits, timing=False, full_space=main_full)
    run("timed", main_bits, full_space=main_full)
    if not args.no_fp32 and main_bits == 64:
        if not args.no_full_space:
            run("fp32_local_full_space", 32, full_space=True)
        run("fp32_local", 32, timing=False)
        run("fp32_local_timed", 32)
    if not args.no_full_space:
        run("full_space", main_bits, full_space=True)
    if not args.no_graph:
        run("graph", main_bits, use_graph=True, timing=False)
    if not args.no_rho:
        run("rho_scaling", main_bits, timing=False, rho_scaling=True)
    if not args.no_coarse_cg:
        run("coarse_cg", main_bits, timing=False, coarse_cg=True)

    def factor_roofline(r, bits):
        """The setup's batched local Cholesky (MFMA-bound): its envelope flops over
        its stream-event time, against the dense MFMA peak of its precision (the
        interface form factors in FP64 for either local precision)."""
        fp32_factors = bits == 32 and r["full_space"]
        peak = 157.3 if fp32_factors else 78.6
        ach = r["factor_flops"] / (r["factor_ms"] * 1e-3) / 1e12 if r["factor_ms"] > 0 else None
        return {"bound": "mfma", "achieved": round(ach, 2) if ach else None, "peak": peak, "unit": "TFLOP/s",
                "frac": round(ach / peak, 4) if ach else None, "flops": r["factor_flops"],
                "ms": round(r["factor_ms"], 3), "dtype": "f32" if fp32_factors else "f64"}

    def summarize(r, bits):
        # element size of each family's matrices: the interface form keeps FP64
        # factors (interior passes) and an FP64 operator whatever local_bits is
        lb = 8 if bits == 64 else 4
        algo = algorithmic_bytes(w, lb, r["env"])
        if not r["full_space"]:
            a8 = algorithmic_bytes(w, 8, r["env"])
            algo["trsv_fwd_ii"], algo["trsv_bwd_ii"] = a8["trsv_fwd_ii"], a8["trsv_bwd_ii"]
        fams = {f: r["kernels"][f] for f in r["families"]}
        out = {"value": round(args.steps / r["elapsed_s"], 3), "unit": "solves/s",
               "ms_per_step": round(1000 * r["elapsed_s"] / args.steps, 3), "iters": r["iters"][-1],
               "relres_true": r["info"]["relres_true"], "cond_est": r["info"]["cond_est"],
               "err_vs_oracle": r["err_vs_oracle"], "setup_s": round(r["setup_s"], 3),
               "dev_bytes": r["dev_bytes"], "autotune": r["tuning"]}
        if not any(v[0] for v in fams.values()):
            return out
        main_fams = FULL_FAMILIES if r["full_space"] else IFACE_FAMILIES
        dom = max(main_fams, key=lambda f: fams[f][1])
        n_l, tot_ms = fams[dom]
        avg_s = tot_ms / 1000.0 / max(n_l, 1)
        achieved = algo[dom] / avg_s / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "frac_of_copy": round(achieved / copy_gbs, 4) if copy_gbs else None,
                "frac_of_read": round(achieved / read_gbs, 4) if read_gbs else None,
                "traffic": load_traffic(dom, args.workload, bits),
                "bytes_per_launch": algo[dom], "avg_launch_ms": round(avg_s * 1e3, 4), "launches": n_l}
        # bytes every family streams per solve (launch counts of the timed run)
        solve_bytes = sum(algo[f] * fams[f][0] for f in r["families"]) / args.steps
        fam_rates = {f: round(algo[f] / (fams[f][1] / 1e3 / fams[f][0]) / 1e9 / HBM_PEAK_GBS, 4)
                     for f in r["families"] if fams[f][0]}
        n_a, ms_a = r["kernels"]["apply"]
        out.update({
            "applies_per_s": round(n_a / (ms_a / 1e3), 2) if n_a else None,
            "kernel_ms": {f: round(fams[f][1] / max(fams[f][0], 1), 4) for f in fams},
            "launches_per_solve": {f: fams[f][0] / args.steps for f in fams},
            "kernel_hbm_frac": fam_rates,
            "bytes_per_solve": int(solve_bytes),
            # the streams of every family over the whole solve time (timed run)
            "solve_hbm_frac": round(solve_bytes / (r["elapsed_s"] / args.steps) / 1e9 / HBM_PEAK_GBS, 4),
            "roofline": roof})
        return out

    m = summarize(runs["main"], main_bits)
    out = {
        "metric": "BDDC-PCG solves/s to rtol 1e-8 (FP64 vs FP32-local) + % HBM/MFMA peak",
        "value": m["value"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_bits == 64 else "f64-outer/f32-local",
        "data": "synthetic",
        "config": {"workload": w.name, "n_free": w.n_free, "subdomains": int(np.prod(w.nsub)),
                   "rtol": w.rtol, "local_bits": main_bits,
                   "cg_space": "whole space" if main_full else "interface", "launch": "eager"},
    }
    for k in ["iters", "relres_true", "cond_est", "err_vs_oracle", "setup_s", "dev_bytes", "autotune"]:
        out[k] = m[k]
    out["timed"] = timed = summarize(runs["timed"], main_bits)
    out["roofline_measured_in"] = "timed run: the same solves with dispatch-recorded events around the kernels"
    out["stream_bandwidth"] = None if copy_gbs is None else {
        "copy_GBps": round(copy_gbs, 1), "read_GBps": round(read_gbs, 1),
        "how": "PyTorch's 1 GiB FP64 device-to-device copy (bytes read plus written per second) and its sum "
               "of the same vector (bytes read per second), median of 5 each: reference points, not ceilings; "
               "roofline.frac_of_copy and frac_of_read are achieved over these"}
    for k in ["applies_per_s", "kernel_ms", "kernel_hbm_frac", "bytes_per_solve", "solve_hbm_frac"]:
        out[k] = timed[k]
    out["roofline"] = timed["roofline"]
    out["setup_factor_roofline"] = factor_roofline(runs["main"], main_bits)
    if "fp32_local" in runs or "fp32_local_full_space" in runs:
        f = {}
        if "fp32_local_full_space" in runs:
            # the FP32-local form as the workload defines it: FP32 local Cholesky
            # factors and triangular solves, FP64 outer CG, r1 and coarse problem
            f = summarize(runs["fp32_local_full_space"], 32)
            f["cg_space"] = "whole space"
            f["local_precision"] = "FP32 local Cholesky factors and triangular solves (MFMA f32)"
            f["setup_factor_roofline"] = factor_roofline(runs["fp32_local_full_space"], 32)
            f["speedup_vs_fp64_full_space"] = None
        if "fp32_local" in runs:
            v = summarize(runs["fp32_local"], 32)
            v["cg_space"] = "interface"
            v["local_precision"] = "FP32 preconditioner matrices (FP64 factors, operator and interior solves)"
            v["timed"] = summarize(runs["fp32_local_timed"], 32)
            for k in ["applies_per_s", "kernel_ms", "kernel_hbm_frac", "solve_hbm_frac", "roofline"]:
                v[k] = v["timed"].get(k)
            v["speedup_vs_fp64"] = round(v["value"] / m["value"], 4)
            f["interface_variant"] = v
        out["fp32_local"] = f
    if "full_space" in runs:
        out["full_space"] = summarize(runs["full_space"], main_bits)
        out["full_space"]["setup_factor_roofline"] = factor_roofline(runs["full_space"], main_bits)
        if out.get("fp32_local", {}).get("value"):
            out["fp32_local"]["speedup_vs_fp64_full_space"] = round(
                out["fp32_local"]["value"] / out["full_space"]["value"], 4)
    if "graph" in runs:
        out["graph"] = summarize(runs["graph"], main_bits)
    if "rho_scaling" in runs:
        out["rho_scaling"] = summarize(runs["rho_scaling"], main_bits)
        out["rho_scaling"]["weights"] = "rho-scaling (coefficient-aware; the paper fixes 1/kappa)"
    if "coarse_cg" in runs:
        out["coarse_cg"] = summarize(runs["coarse_cg"], main_bits)
        out["coarse_cg"]["coarse_solve"] = "Jacobi-preconditioned CG to 1e-13 (the paper's choice) at every apply"
    if not args.no_secondary and args.workload != "3d_64":
        w64 = W.cfg_3d_64()
        r64 = run_gpu(w64, args.steps, args.warmup, main_bits, timing=False, golden=load_golden("3d_64"))
        out["secondary_3d_64"] = {"workload": w64.name, "value": round(args.steps / r64["elapsed_s"], 3),
                                  "unit": "solves/s", "ms_per_step": round(1000 * r64["elapsed_s"] / args.steps, 3),
                                  "iters": r64["iters"][-1], "relres_true": r64["info"]["relres_true"],
                                  "err_vs_oracle": r64["err_vs_oracle"]}
        print(f"[bench] secondary 3d_64: {1000 * r64['elapsed_s'] / args.steps:.2f} ms/solve", file=sys.stderr,
              flush=True)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_report()
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, m["iters"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
