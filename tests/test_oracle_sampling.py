"""CPU: the oracle's stochastic viewgraph sub-sampling (counter-based
SplitMix64 keys, min(|E|, M) image pairs per scene, both directions of a pair
together) and the loss of a sub-sampled step."""
import os

import numpy as np
import pytest

from oracle import cost, sampling
from synth import fixtures, make
from synth.scenes import pack

HERE = os.path.dirname(os.path.abspath(__file__))


def test_splitmix64_reference_outputs():
    """The generator reproduces published SplitMix64 outputs (state advanced
    by the golden gamma before each output)."""
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "splitmix64.txt"))
            if l.strip() and not l.startswith("#")]
    assert rows
    for row in rows:
        seed, want = int(row[0]), [int(x) for x in row[1:]]
        got = [sampling.splitmix64((seed + k * sampling.GOLDEN_GAMMA) & sampling.MASK)
               for k in range(len(want))]
        assert got == want


def test_pair_groups_pair_both_directions():
    pairs = np.array([[0, 1], [1, 0], [2, 0], [1, 2], [0, 2], [3, 1]])
    g, n = sampling.pair_groups(pairs)
    assert n == 4
    assert list(g) == [0, 0, 1, 2, 1, 3]


@pytest.mark.parametrize("budget", [1, 5, 28, 100])
def test_subset_size_and_directions(budget):
    p = make("c2")                       # 28 image pairs, both directions each
    for step in range(5):
        sel = sampling.selected_pairs(p.pairs, p.scene_of_pair, 7, step, budget)
        g, n = sampling.pair_groups(p.pairs)
        chosen = np.unique(g[sel])
        assert chosen.size == min(n, budget)
        # a pair is selected iff its reverse is
        assert np.array_equal(np.sort(g[sel]), np.sort(np.repeat(chosen, 2)))


def test_subsets_are_fresh_each_step_and_reproducible():
    p = make("c2")
    a = [sampling.selected_pairs(p.pairs, p.scene_of_pair, 3, s, 10) for s in range(6)]
    b = [sampling.selected_pairs(p.pairs, p.scene_of_pair, 3, s, 10) for s in range(6)]
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert len({x.tobytes() for x in a}) == 6
    c = sampling.selected_pairs(p.pairs, p.scene_of_pair, 4, 0, 10)
    assert not np.array_equal(a[0], c)


def test_selection_is_uniform_over_pairs():
    """Every image pair is drawn with frequency M/|E| (binomial bounds over
    2000 steps), and per-step subset sizes are exact."""
    group_scene = np.zeros(28, np.int64)
    steps, M = 2000, 7
    counts = np.zeros(28)
    for s in range(steps):
        sel = sampling.select_groups(group_scene, 11, s, M)
        assert sel.sum() == M
        counts += sel
    p = M / 28
    sd = np.sqrt(steps * p * (1 - p))
    assert np.abs(counts - steps * p).max() < 5 * sd
    # pairwise co-selection also matches a uniform M-subset
    chi = ((counts - steps * p) ** 2 / (steps * p)).sum()
    assert chi < 27 + 6 * np.sqrt(2 * 27)


def test_selection_per_scene():
    """Each scene draws its own min(|E_scene|, M) pairs."""
    p1 = make("c1")
    p2 = make("c2")
    both = pack(list(p2.scenes) + list(p1.scenes), "two")
    for step in range(3):
        sel = sampling.selected_pairs(both.pairs, both.scene_of_pair, 5, step, 4)
        g, _ = sampling.pair_groups(both.pairs)
        for s, n_groups in ((0, 28), (1, 1)):
            mine = np.unique(g[sel & (both.scene_of_pair == s)])
            assert mine.size == min(4, n_groups)


def test_subsampled_loss_is_the_mean_over_selected_pairs():
    p = make("c2")
    op = cost.OracleProblem(p)
    full = op.evaluate(p.poses_init, 10.0)
    sel = sampling.selected_pairs(p.pairs, p.scene_of_pair, 1, 0, 9)
    r = op.evaluate(p.poses_init, 10.0, selected=sel)
    assert sel.sum() == 18
    # (2/|D_S|) sum of L_d = (1/|E_S|) sum over the selected image pairs of
    # (L_ij + L_ji)
    np.testing.assert_allclose(r["loss"], [2.0 * full["L"][sel].mean()], rtol=1e-14)
    # per-pair quantities of the selected pairs are the full evaluation's
    np.testing.assert_array_equal(r["S"][sel], full["S"][sel])
    assert np.all(r["w"][~sel] == 0)
    # every pair selected: identical to the full evaluation
    r_all = op.evaluate(p.poses_init, 10.0, selected=np.ones(p.pairs.shape[0], bool))
    np.testing.assert_array_equal(r_all["loss"], full["loss"])
    np.testing.assert_array_equal(r_all["grad"], full["grad"])


def test_subset_gradient_is_unbiased():
    """Averaged over every subset of size M of a scene's image pairs (here all
    C(4, 2) = 6 two-pair subsets of a 4-view scene), the sub-sampled loss
    and gradient equal the full-graph ones."""
    from itertools import combinations
    p = make("c2")
    q = fixtures.problem_from_maps(p.width[:4], p.height[:4], p.K[:4],
                                   [p.edge_map(v) for v in range(4)],
                                   [p.depth_map(v) for v in range(4)], p.poses_init[:4],
                                   [(a, b) for a in range(4) for b in range(4) if a < b],
                                   name="sub4")
    q_pairs = np.concatenate([q.pairs, q.pairs[:, ::-1]])
    q2 = fixtures.problem_from_maps(q.width, q.height, q.K, [q.edge_map(v) for v in range(4)],
                                    [q.depth_map(v) for v in range(4)], q.poses_init,
                                    [tuple(x) for x in q_pairs], name="sub4b")
    op = cost.OracleProblem(q2)
    full = op.evaluate(q2.poses_init, 10.0)
    g, n = sampling.pair_groups(q2.pairs)
    loss, grad, k = 0.0, 0.0, 0
    for subset in combinations(range(n), 2):
        sel = np.isin(g, subset)
        r = op.evaluate(q2.poses_init, 10.0, selected=sel)
        loss = loss + r["loss"]
        grad = grad + r["grad"]
        k += 1
    np.testing.assert_allclose(loss / k, full["loss"], rtol=1e-12)
    np.testing.assert_allclose(grad / k, full["grad"], rtol=1e-10, atol=1e-14)
