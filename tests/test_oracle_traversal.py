"""Pin of the oracle's cell traversal (Sec. 2.1: the length Delta r between two
consecutive cell interfaces crossed by a ray) against brute-force ray-box
intersection lengths on tiny grids."""
import numpy as np
import pytest


def slab_interval(xs, n, lo, hi):
    """[t0, t1] of the ray xs + t n inside the box [lo, hi] (may be empty)."""
    t0, t1 = -np.inf, np.inf
    for a in range(3):
        if n[a] != 0.0:
            ta = (lo[a] - xs[a]) / n[a]
            tb = (hi[a] - xs[a]) / n[a]
            t0 = max(t0, min(ta, tb))
            t1 = min(t1, max(ta, tb))
        elif not (lo[a] <= xs[a] < hi[a]):
            return 1.0, 0.0
    return t0, t1


def brute_lengths(shape, xs, n, r_a, r_end):
    nx, ny, nz = shape
    t0, t1 = slab_interval(xs, n, (0, 0, 0), (nx, ny, nz))
    r_end = min(r_end, t1)
    out = {}
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                a, b = slab_interval(xs, n, (i, j, k), (i + 1, j + 1, k + 1))
                length = min(b, r_end) - max(a, r_a)
                if length > 0:
                    out[(k * ny + j) * nx + i] = length
    return out


@pytest.mark.parametrize("seed", range(6))
def test_segments_match_brute_force(oracle, seed):
    rng = np.random.default_rng(seed)
    shape = (5, 6, 4)
    for _ in range(150):
        xs = rng.uniform(0, 1, 3) * np.array(shape)
        n = rng.standard_normal(3)
        if seed == 0:  # rays along axes and diagonals exercise ties
            n = np.array(rng.choice([-1.0, 0.0, 1.0], size=3))
            if not n.any():
                n[0] = 1.0
        n /= np.linalg.norm(n)
        r_a = rng.uniform(0, 2)
        r_end = r_a + rng.uniform(0, 8)
        cells, drs = oracle.ray_segments(shape, xs, n, r_a, r_end)
        got = {}
        for c, d in zip(cells, drs):
            got[int(c)] = got.get(int(c), 0.0) + d
        want = brute_lengths(shape, xs, n, r_a, r_end)
        for c in set(got) | set(want):
            assert got.get(c, 0.0) == pytest.approx(want.get(c, 0.0), abs=1e-12)
        t0, t1 = slab_interval(xs, n, (0, 0, 0), shape)
        total = max(0.0, min(r_end, t1) - r_a)
        assert drs.sum() == pytest.approx(total, abs=1e-12)
        assert (drs > 0).all()


def test_consecutive_cells_are_face_neighbours(oracle):
    rng = np.random.default_rng(7)
    shape = (16, 16, 16)
    for _ in range(50):
        xs = rng.uniform(0, 16, 3)
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        cells, _ = oracle.ray_segments(shape, xs, n, 0.0, 100.0)
        ijk = np.stack([cells % 16, (cells // 16) % 16, cells // 256], 1)
        step = np.abs(np.diff(ijk, axis=0)).sum(1)
        assert (step >= 1).all() and (step <= 3).all()
