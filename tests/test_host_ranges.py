"""Host checks of the range arithmetic the interface mat-vec relies on (no GPU):
the launch gives workgroup g of G the tiles [floor(g N / G), floor((g+1) N / G)),
the finishing kernels recover the workgroup of tile p as
floor(((p + 1) G - 1) / N), and they divide by one FP64 division, which is exact
after flooring whenever a + b < 2^53."""
import random

import pytest


def ranges(n, g):
    return [(k * n // g, (k + 1) * n // g) for k in range(g)]


def wg_of(p, n, g):
    return ((p + 1) * g - 1) // n


@pytest.mark.parametrize("n,g", [(10, 4), (141308, 512), (141308, 768), (7, 7), (1536, 256), (1000003, 4096)])
def test_workgroup_of_tile_inverts_the_split(n, g):
    rs = ranges(n, g)
    rng = random.Random(n * 31 + g)
    ps = set(rng.randrange(n) for _ in range(2000)) | {0, n - 1} | {a for a, b in rs if a < n}
    for p in ps:
        k = wg_of(p, n, g)
        a, b = rs[k]
        assert a <= p < b, (p, k, a, b)


def test_first_slot_rule_matches_a_direct_walk():
    """A column's slot holds a sum exactly when it is the column's first tile in
    its workgroup's range: walk the packed lower tile triangle of a few matrices
    in stream order and compare with the rule used by the finishing kernels."""
    rng = random.Random(5)
    ts_list = [rng.randrange(1, 30) for _ in range(12)]
    tri = lambda i, j: i * (i + 1) // 2 + j
    n = sum(t * (t + 1) // 2 for t in ts_list)
    for g in (1, 3, 17, 64, n):
        first_seen = set()
        off = 0
        for ts in ts_list:
            seen = {}
            for i in range(ts):
                for j in range(i + 1):
                    p = off + tri(i, j)
                    key = (wg_of(p, n, g), j)
                    if key not in seen:
                        seen[key] = p
            first_seen |= set(seen.values())
            for j in range(ts):
                for i in range(j, ts):
                    p = off + tri(i, j)
                    rule = i == j or wg_of(p, n, g) != wg_of(off + tri(i - 1, j), n, g)
                    assert rule == (p in first_seen), (g, ts, i, j)
            off += ts * (ts + 1) // 2


def test_one_fp64_division_floors_exactly():
    rng = random.Random(11)
    cases = [(a, b) for a, b in [(0, 1), (2**40, 3), (2**52 - 7, 5), (141308 * 4096, 141308)]]
    for _ in range(20000):
        b = rng.randrange(1, 1 << rng.randrange(1, 40))
        a = rng.randrange(0, (1 << 53) - b)
        cases.append((a, b))
        k = rng.randrange(0, ((1 << 53) - 1) // (b + 1)) if b < (1 << 26) else 0
        cases.append((k * b + b - 1, b))   # just below a multiple: the worst case
    for a, b in cases:
        if a + b >= 1 << 53:
            continue
        assert int(float(a) / float(b)) == a // b, (a, b)
