"""GPU: the viewgraph entry point that allocates nothing
(epo_build_viewgraph_noalloc, staging in a static device array) against the
allocating epo_build_viewgraph, through the C-ABI: consistent and total
counts and validity flags bitwise equal, on two calls in a row, the second
with fewer views, fewer candidates and a coarser grid (the static array keeps
the first call's contents)."""
import numpy as np
import pytest
import torch

from synth.dense import dense_depth
from tests.gpu_helpers import problem, say

pytestmark = pytest.mark.gpu


def run(fn, p, depth, poses, stride):
    from paper_2607_00579_amd.api import _stream
    dev = torch.device("cuda:0")
    sov = np.asarray(p.scene_of_view, np.int64)
    iu, ju = np.triu_indices(p.n_views, 1)
    same = sov[iu] == sov[ju]
    cand = np.ascontiguousarray(np.stack([iu[same], ju[same]], axis=1).astype(np.int32))
    n = cand.shape[0]
    # outputs start as garbage: the call must write every entry
    cons = torch.full((n,), -7, dtype=torch.int32, device=dev)
    tot = torch.full((n,), -7, dtype=torch.int32, device=dev)
    valid = torch.full((n,), 9, dtype=torch.uint8, device=dev)
    fn(p.n_views, np.ascontiguousarray(p.width, np.int32), np.ascontiguousarray(p.height, np.int32),
       np.ascontiguousarray(p.K, np.float32).reshape(-1, 4),
       np.ascontiguousarray(p.view_offset, np.int64)[:p.n_views], depth, poses, cand, n, stride,
       3.0, 0.125, 1e-4, cons, tot, valid, _stream(dev))
    torch.cuda.synchronize()
    return cons.cpu().numpy(), tot.cpu().numpy(), valid.cpu().numpy()


def test_noalloc_viewgraph_equals_allocating_form(gpu):
    from paper_2607_00579_amd import _lib
    for name, stride in (("c3", 4), ("c2", 6)):
        p = problem(name)
        depth = torch.from_numpy(dense_depth(p, sigma=0.005, seed=1)).cuda()
        poses = torch.from_numpy(np.ascontiguousarray(p.poses_init)).cuda()
        a = run(_lib.build_viewgraph, p, depth, poses, stride)
        b = run(_lib.build_viewgraph_noalloc, p, depth, poses, stride)
        say(f"{name}: {a[0].size} candidates, {int(a[2].sum())} valid; no-allocation form "
            f"equal: {all(np.array_equal(x, y) for x, y in zip(a, b))}")
        assert (a[1] > 0).all() and set(np.unique(a[2])) <= {0, 1}
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
