"""Seeded synthetic workloads for BDDC-preconditioned CG on Q1 diffusion problems.

This module only *draws data*: meshes, box partitions, per-element
conductivities, right-hand sides and finite-difference picks.  It holds none
of the method's arithmetic, so both the CPU oracle and the GPU path may use it.

Conventions (shared by every consumer):
  * unit square / cube, ``nel[a]`` elements along axis ``a``;
  * element (ex, ey, ez) has index ex + nx*(ey + ny*ez) (x fastest);
  * free dofs are the interior nodes, index
    (ix-1) + (nx-1)*((iy-1) + (ny-1)*(iz-1));
  * a partition is a tensor product of cut lists, cuts[a][0] = 0 < ... <
    cuts[a][-1] = nel[a]; box (bx, by, bz) has index bx + Bx*(by + By*bz);
  * seeds: numpy SeedSequence(seed).spawn(4) gives independent streams for
    [cuts, theta, b, fd-picks].

The problem statement these follow is the paper's 2D Poisson setting on the
unit square split into equal square subdomains (Sec. 3), extended to the 3D
diffusion workloads and coefficient fields listed below.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

CORNERS = 1
EDGES = 2
FACES = 4
ALL_PRIMAL = 8


@dataclasses.dataclass
class Workload:
    name: str
    dim: int
    nel: Tuple[int, ...]
    cuts: List[np.ndarray]           # per axis, int64, first 0, last nel[a]
    theta: np.ndarray                # float64, n_el, element order x fastest
    b: np.ndarray                    # float64, n_free
    constraints: int
    rtol: float
    local_bits: int = 64
    theta_obs: Optional[np.ndarray] = None   # adjoint workload only
    fd_elements: Optional[np.ndarray] = None  # adjoint workload only
    seed: int = 0

    @property
    def n_el(self) -> int:
        return int(np.prod(self.nel))

    @property
    def n_free(self) -> int:
        return int(np.prod([n - 1 for n in self.nel]))

    @property
    def nsub(self) -> Tuple[int, ...]:
        return tuple(len(c) - 1 for c in self.cuts)


def _streams(seed: int):
    ss = np.random.SeedSequence(seed).spawn(4)
    return [np.random.default_rng(s) for s in ss]


def uniform_cuts(nel: int, nsub: int) -> np.ndarray:
    """Equal boxes; nel must be divisible by nsub."""
    if nel % nsub:
        raise ValueError(f"{nel} elements cannot be split into {nsub} equal boxes")
    return np.arange(0, nel + 1, nel // nsub, dtype=np.int64)


def random_cuts(rng: np.random.Generator, nel: int, nsub: int, lo: int, hi: int) -> np.ndarray:
    """Box lengths drawn uniformly in [lo, hi] per box, redrawn until they sum to nel."""
    if not (nsub * lo <= nel <= nsub * hi):
        raise ValueError("no admissible lengths")
    while True:
        lens = rng.integers(lo, hi + 1, size=nsub)
        if int(lens.sum()) == nel:
            return np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)


def lognormal_theta(rng: np.random.Generator, n_el: int) -> np.ndarray:
    return np.exp(rng.standard_normal(n_el))


def inclusion_theta(rng: np.random.Generator, nel: Sequence[int], cuts: Sequence[np.ndarray],
                    inside: float = 1e-3, outside: float = 1.0) -> np.ndarray:
    """One axis-aligned ellipsoid per box: centre = box centre + U(-.05,.05)*dims,
    semi-axes U(.2,.4)*dims; an element is inside iff its centroid is."""
    dim = len(nel)
    nsub = [len(c) - 1 for c in cuts]
    theta = np.full(int(np.prod(nel)), outside, dtype=np.float64)
    # element centroids per axis
    cent = [np.arange(n) + 0.5 for n in nel]
    for bidx in range(int(np.prod(nsub))):
        bc = []
        r = bidx
        for a in range(dim):
            bc.append(r % nsub[a])
            r //= nsub[a]
        lo = np.array([cuts[a][bc[a]] for a in range(dim)], dtype=np.float64)
        hi = np.array([cuts[a][bc[a] + 1] for a in range(dim)], dtype=np.float64)
        dims = hi - lo
        centre = 0.5 * (lo + hi) + rng.uniform(-0.05, 0.05, size=dim) * dims
        semi = rng.uniform(0.2, 0.4, size=dim) * dims
        ranges = [np.arange(int(lo[a]), int(hi[a])) for a in range(dim)]
        grids = np.meshgrid(*ranges, indexing="ij")
        q = np.zeros(grids[0].shape)
        for a in range(dim):
            q += ((cent[a][grids[a]] - centre[a]) / semi[a]) ** 2
        inside_mask = q <= 1.0
        eidx = np.zeros(grids[0].shape, dtype=np.int64)
        stride = 1
        for a in range(dim):
            eidx += grids[a] * stride
            stride *= nel[a]
        theta[eidx[inside_mask]] = inside
    return theta


def make_workload(name: str, dim: int, nel: Sequence[int], nsub: Sequence[int] = None,
                  cuts: Sequence[np.ndarray] = None, theta: str = "one",
                  constraints: Optional[int] = None, rtol: float = 1e-8, seed: int = 0,
                  local_bits: int = 64, random_box: Tuple[int, int] = None) -> Workload:
    """Generic seeded workload (tests use small ones; the named configs below use this)."""
    nel = tuple(int(n) for n in nel)
    rc, rt, rb, rf = _streams(seed)
    if cuts is None:
        if random_box is not None:
            cuts = [random_cuts(rc, nel[a], nsub[a], *random_box) for a in range(dim)]
        else:
            cuts = [uniform_cuts(nel[a], nsub[a]) for a in range(dim)]
    cuts = [np.asarray(c, dtype=np.int64) for c in cuts]
    n_el = int(np.prod(nel))
    if theta == "one":
        th = np.ones(n_el)
    elif theta == "lognormal":
        th = lognormal_theta(rt, n_el)
    elif theta == "inclusions":
        th = inclusion_theta(rt, nel, cuts)
    else:
        raise ValueError(theta)
    n_free = int(np.prod([n - 1 for n in nel]))
    b = rb.uniform(-1.0, 1.0, n_free)
    if constraints is None:
        constraints = CORNERS | EDGES | (FACES if dim == 3 else 0)
    return Workload(name=name, dim=dim, nel=nel, cuts=cuts, theta=th, b=b,
                    constraints=constraints, rtol=rtol, local_bits=local_bits, seed=seed)


def cfg_2d_64(seed: int = 0) -> Workload:
    """2D Q1, 64x64 elements, 4x4 boxes of 16x16, theta = 1, corners + edge
    averages, FP64 to relative residual 1e-10."""
    return make_workload("2d_q1_64x64_4x4_theta1", 2, (64, 64), (4, 4), theta="one",
                         constraints=CORNERS | EDGES, rtol=1e-10, seed=seed)


def cfg_3d_64(seed: int = 0, local_bits: int = 64) -> Workload:
    """3D Q1, 64^3 elements, 4^3 boxes of 16^3, lognormal(0,1) theta, corners +
    edge + face averages, rtol 1e-8."""
    return make_workload("3d_q1_64cubed_4x4x4_lognormal", 3, (64, 64, 64), (4, 4, 4),
                         theta="lognormal", rtol=1e-8, seed=seed, local_bits=local_bits)


def cfg_3d_128_uneven(seed: int = 0, local_bits: int = 64) -> Workload:
    """3D Q1, 128^3 elements, 8^3 tensor boxes with lengths drawn in [8, 24],
    one 1e-3 ellipsoid inclusion per box, rtol 1e-8."""
    return make_workload("3d_q1_128cubed_512_uneven_inclusions", 3, (128, 128, 128), (8, 8, 8),
                         theta="inclusions", rtol=1e-8, seed=seed, local_bits=local_bits,
                         random_box=(8, 24))


def cfg_3d_96_adjoint(seed: int = 0, n_fd: int = 16) -> Workload:
    """3D Q1, 96^3 elements, 6^3 boxes of 16^3, lognormal theta; the observed
    field comes from theta_obs = theta*exp(0.1 Z'); FP32-local factors."""
    w = make_workload("3d_q1_96cubed_6x6x6_adjoint", 3, (96, 96, 96), (6, 6, 6),
                      theta="lognormal", rtol=1e-8, seed=seed, local_bits=32)
    add_adjoint_data(w, n_fd)
    return w


def add_adjoint_data(w: Workload, n_fd: int = 16) -> None:
    """theta_obs = theta*exp(0.1 Z') and n_fd distinct element picks, from the
    fourth seed stream."""
    rf = _streams(w.seed)[3]
    w.theta_obs = w.theta * np.exp(0.1 * rf.standard_normal(w.n_el))
    w.fd_elements = np.sort(rf.choice(w.n_el, size=min(n_fd, w.n_el), replace=False)).astype(np.int64)


def cfg_3d_128_uneven_fp32(seed: int = 0) -> Workload:
    """The 128^3 uneven-box workload with FP32 local factors and solves."""
    return cfg_3d_128_uneven(seed, local_bits=32)


WORKLOADS = {
    "2d_64": cfg_2d_64,
    "3d_64": cfg_3d_64,
    "3d_128_uneven": cfg_3d_128_uneven,
    "3d_128_uneven_fp32": cfg_3d_128_uneven_fp32,
    "3d_96_adjoint": cfg_3d_96_adjoint,
}
