"""Pins of the oracle's exact distance transform (CPU)."""
import numpy as np
import pytest

from oracle import edt

INF = edt.INF_D2


def all_4x4_maps():
    m = np.arange(1 << 16, dtype=np.int64)
    bits = ((m[:, None] >> np.arange(16)[None, :]) & 1).astype(bool)   # (65536, 16), pixel p = 4 y + x
    return bits


def brute_all_4x4(bits):
    ys, xs = np.divmod(np.arange(16), 4)
    dist = (xs[:, None] - xs[None, :]) ** 2 + (ys[:, None] - ys[None, :]) ** 2   # (p, q)
    out = np.empty(bits.shape, np.int64)
    for p in range(16):
        out[:, p] = np.where(bits, dist[p][None, :], INF).min(axis=1)
    return out


def test_exhaustive_4x4_separable_matches_definition():
    bits = all_4x4_maps()
    ref = brute_all_4x4(bits)
    for k in range(bits.shape[0]):
        e = bits[k].reshape(4, 4).astype(np.uint8)
        assert np.array_equal(edt.edt_separable(e).reshape(-1), ref[k]), k


def test_4x4_fh_matches_definition_on_sample():
    bits = all_4x4_maps()
    ref = brute_all_4x4(bits)
    rng = np.random.default_rng(0)
    for k in np.concatenate([[0, 1, 65535], rng.integers(0, 1 << 16, 3000)]):
        e = bits[k].reshape(4, 4).astype(np.uint8)
        assert np.array_equal(edt.edt_fh(e).reshape(-1), ref[k]), k


@pytest.mark.parametrize("shape", [(1, 17), (17, 1), (33, 17), (48, 64), (7, 5)])
@pytest.mark.parametrize("density", [0.001, 0.01, 0.1, 0.5])
def test_random_maps_three_ways(shape, density):
    rng = np.random.default_rng(hash((shape, density)) % (1 << 32))
    e = (rng.random(shape) < density).astype(np.uint8)
    a = edt.edt_bruteforce(e)
    assert np.array_equal(a, edt.edt_fh(e))
    assert np.array_equal(a, edt.edt_separable(e))


def test_single_pixel_closed_form():
    H, W = 23, 31
    for (y0, x0) in [(0, 0), (11, 17), (22, 30), (5, 0)]:
        e = np.zeros((H, W), np.uint8)
        e[y0, x0] = 1
        yy, xx = np.mgrid[0:H, 0:W]
        want = (xx - x0) ** 2 + (yy - y0) ** 2
        assert np.array_equal(edt.edt_fh(e), want)
        assert np.array_equal(edt.edt_separable(e), want)


def test_empty_and_full():
    e = np.zeros((6, 9), np.uint8)
    for f in (edt.edt_bruteforce, edt.edt_fh, edt.edt_separable):
        assert (f(e) == INF).all()
        assert (f(np.ones_like(e)) == 0).all()


def test_column_map_closed_form():
    H, W, c = 12, 20, 7
    e = np.zeros((H, W), np.uint8)
    e[:, c] = 1
    want = np.broadcast_to((np.arange(W) - c) ** 2, (H, W))
    assert np.array_equal(edt.edt_separable(e), want)
    assert np.array_equal(edt.edt_fh(e), want)


def test_lower_envelope_1d_bruteforce():
    rng = np.random.default_rng(5)
    for _ in range(300):
        n = int(rng.integers(1, 40))
        f = [None if rng.random() < 0.4 else int(rng.integers(0, 400)) for _ in range(n)]
        got = edt.lower_envelope_1d(f)
        fin = [(p, fp) for p, fp in enumerate(f) if fp is not None]
        for q in range(n):
            want = min((fp + (q - p) ** 2 for p, fp in fin), default=None)
            assert got[q] == want


def test_row_minimizers_are_monotone():
    """The property the GPU row pass rests on (brute force, no oracle code):
    for g(x) = min over q of f(q) + (x - q)^2 and X0 < x < X1, some minimizer
    of x lies between any minimizer of X0 and any minimizer of X1, so the
    minimum over that range equals g(x).  Random rows with ties, empty
    stretches (a large f) and single small values."""
    rng = np.random.default_rng(5)
    big = 1 << 30
    for trial in range(300):
        W = int(rng.integers(2, 80))
        f = rng.integers(0, 40, W) ** 2
        f[rng.random(W) < rng.random()] = big
        x = np.arange(W)
        cost = f[None, :] + (x[:, None] - x[None, :]) ** 2       # [x, q]
        g = cost.min(axis=1)
        for _ in range(10):
            X0, X1 = sorted(rng.choice(W, 2, replace=False))
            for qa in np.flatnonzero(cost[X0] == g[X0]):
                for qb in np.flatnonzero(cost[X1] == g[X1]):
                    assert qa <= qb
                    for xx in range(X0 + 1, X1):
                        assert cost[xx, qa:qb + 1].min() == g[xx], (trial, X0, X1, xx)


@pytest.mark.parametrize("S,pitch,x0,y0", [(64, 8, 3, 5), (61, 8, 3, 5), (40, 6, 0, 5), (33, 4, 3, 1)])
def test_grid_closed_form_matches_oracle_edt(S, pitch, x0, y0):
    """The closed-form distance field that the maximum-size GPU test hands the
    oracle (edge pixels on a regular grid: the nearest grid column and row)
    equals the square root of the oracle's exact transform of the same map,
    borders and sides that end between grid lines included."""
    from tests.gpu_helpers import GridDTF
    e = np.zeros((S, S), np.uint8)
    e[y0::pitch, x0::pitch] = 1
    yy, xx = np.mgrid[0:S, 0:S]
    got = GridDTF(S, pitch, x0, y0)[yy, xx]
    assert np.array_equal(got, np.sqrt(edt.edt_separable(e).astype(np.float64)))
