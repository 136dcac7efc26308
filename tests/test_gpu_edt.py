"""GPU: exact distance transform, bit-exact against the oracle."""
import numpy as np
import pytest
import torch

from oracle import edt as oedt
from tests.gpu_helpers import problem, say

pytestmark = pytest.mark.gpu


def gpu_edt(maps):
    """Run the HIP EDT on a list of uint8 maps packed back to back."""
    from paper_2607_00579_amd.api import build_distance_fields
    sizes = [m.size for m in maps]
    off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    flat = np.concatenate([m.reshape(-1) for m in maps]).astype(np.uint8)
    e = torch.from_numpy(flat).cuda()
    d2, dtf = build_distance_fields(e, off, [m.shape[1] for m in maps], [m.shape[0] for m in maps])
    d2 = d2.cpu().numpy()
    dtf = dtf.cpu().numpy()
    return ([d2[o:o + m.size].reshape(m.shape) for o, m in zip(off, maps)],
            [dtf[o:o + m.size].reshape(m.shape) for o, m in zip(off, maps)])


def test_all_4x4_maps_bit_exact(gpu):
    say("edt: all 65536 4x4 maps")
    m = np.arange(1 << 16, dtype=np.int64)
    bits = ((m[:, None] >> np.arange(16)[None, :]) & 1).astype(np.uint8)
    maps = [b.reshape(4, 4) for b in bits]
    got, dtf = gpu_edt(maps)
    ys, xs = np.divmod(np.arange(16), 4)
    dist = (xs[:, None] - xs[None, :]) ** 2 + (ys[:, None] - ys[None, :]) ** 2
    want = np.empty((1 << 16, 16), np.int64)
    for p in range(16):
        want[:, p] = np.where(bits.astype(bool), dist[p][None, :], oedt.INF_D2).min(axis=1)
    got = np.stack([g.reshape(-1) for g in got])
    assert np.array_equal(got, want)
    assert np.array_equal(np.stack([d.reshape(-1) for d in dtf]),
                          np.sqrt(want.astype(np.float32)).astype(np.float32))


@pytest.mark.parametrize("shape", [(1, 1), (1, 37), (37, 1), (33, 17), (120, 160), (97, 301),
                                   (392, 518)])
@pytest.mark.parametrize("density", [0.0, 0.0005, 0.01, 0.1, 0.6, 1.0])
def test_random_maps_bit_exact(gpu, shape, density):
    rng = np.random.default_rng(abs(hash((shape, density))) % (1 << 32))
    maps = [(rng.random(shape) < density).astype(np.uint8) * 255 for _ in range(3)]
    got, _ = gpu_edt(maps)
    for g, m in zip(got, maps):
        assert np.array_equal(g, oedt.edt_separable(m))


def test_wide_and_single_pixel(gpu):
    """Maps with one or two edge pixels: d2 is the closed-form minimum over
    them.  The row pass stages a row, its block, group and super minima and
    the block starts' minimizers in LDS: rows of up to 14508 pixels fit in
    64 KB, wider ones (14509, 15361, 15420, 15500, 16384) need more."""
    cases = [(3, 4000, [(1, 3999)]), (2000, 2, [(0, 0)]), (64, 2048, [(63, 1000)]),
             (2, 16384, [(1, 5)]), (3, 15500, [(0, 15499)]),
             (2, 14508, [(1, 14507)]), (2, 14509, [(0, 7000)]),
             (2, 15360, [(1, 15359)]), (2, 15361, [(0, 7000)]),
             (2, 15420, [(1, 15419)]), (2, 15421, [(0, 7000)]),
             (4, 16384, [(0, 9000), (3, 9100)])]
    maps = []
    for H, W, pts in cases:
        e = np.zeros((H, W), np.uint8)
        for y0, x0 in pts:
            e[y0, x0] = 1
        maps.append(e)
    got, _ = gpu_edt(maps)
    for g, m, (H, W, pts) in zip(got, maps, cases):
        yy, xx = np.mgrid[0:H, 0:W]
        want = np.min([(xx - x0) ** 2 + (yy - y0) ** 2 for y0, x0 in pts], axis=0)
        assert np.array_equal(g, want), (H, W)


def test_sparse_wide_rows_closed_form(gpu):
    """Few edge pixels in wide rows, the case the row pass's group (256 px)
    and super (4096 px) minima are for: edges on and next to those
    boundaries, at both ends of a 16384-pixel row, and a few random pixels
    per map; d2 is the closed-form minimum over the edge pixels."""
    rng = np.random.default_rng(11)
    cases = [(2, 16384, [(0, 0), (1, 16383)]), (3, 9000, [(2, 255)]), (3, 9000, [(0, 256)]),
             (2, 12289, [(0, 4095), (1, 4096)]), (5, 8192, [(4, 8191)]), (1, 16384, [(0, 8192)])]
    for _ in range(8):
        H, W = int(rng.integers(1, 9)), int(rng.integers(4000, 16385))
        n = int(rng.integers(1, 6))
        cases.append((H, W, [(int(rng.integers(0, H)), int(rng.integers(0, W))) for _ in range(n)]))
    maps = []
    for H, W, pts in cases:
        e = np.zeros((H, W), np.uint8)
        for y0, x0 in pts:
            e[y0, x0] = 1
        maps.append(e)
    got, _ = gpu_edt(maps)
    for g, (H, W, pts) in zip(got, cases):
        yy, xx = np.mgrid[0:H, 0:W]
        want = np.min([(xx - x0) ** 2 + (yy - y0) ** 2 for y0, x0 in pts], axis=0)
        assert np.array_equal(g, want), (H, W, pts)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_config_maps_bit_exact(gpu, name):
    p = problem(name)
    maps = [p.edge_map(v) for v in range(p.n_views)]
    say(f"edt: {name} {len(maps)} views")
    got, _ = gpu_edt(maps)
    for v, (g, m) in enumerate(zip(got, maps)):
        assert np.array_equal(g, oedt.edt_separable(m)), v
