"""Oracle: stochastic viewgraph sub-sampling (paper supplementary Sec.
"Stochastic viewgraph sub-sampling"; Alg. EPO.Forward, pair budget M).

Test infrastructure only (see the package header).

At every optimization step the loss is evaluated on a fresh uniform random
subset of the viewgraph's image pairs, of size min(|E|, M) (default M = 1024),
drawn per scene.  An image pair is an unordered pair {i, j}; the directions of
it that the directed pair list holds are evaluated together, and the loss is
the mean over the evaluated directions (L = (2/|D_S|) sum_{d in D_S} L_d with
D_S the selected directed pairs of the scene), so each step's loss and
gradient are unbiased estimates of the full-graph ones.

The draw is made reproducible across the device and this oracle with a
counter-based generator, SplitMix64 (G. L. Steele, D. Lea, C. H. Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014), whose output
function for a 64-bit state x is

    z = x + 0x9E3779B97F4A7C15
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    h(x) = z ^ (z >> 31)                      (all arithmetic mod 2^64)

Group g of the scene gets the key k(seed, step, g) = h(h(seed + step) + g), and
the selected groups are the min(|E_scene|, M) groups with the smallest
(key, g).  Keys of distinct groups behave as independent uniform draws, so
every subset of that size is equally likely.
"""
from __future__ import annotations

import numpy as np

MASK = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15


def splitmix64(x: int) -> int:
    """SplitMix64 output for state x (the first output of a generator seeded
    with x)."""
    z = (x + GOLDEN_GAMMA) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def group_key(seed: int, step: int, group: int) -> int:
    return splitmix64((splitmix64((seed + step) & MASK) + group) & MASK)


def pair_groups(pairs: np.ndarray):
    """Unordered image pair of every directed pair: group ids numbered in
    order of first appearance in the list."""
    ids = {}
    group_of_pair = np.empty(len(pairs), np.int64)
    for d, (i, j) in enumerate(np.asarray(pairs, np.int64)):
        key = (min(int(i), int(j)), max(int(i), int(j)))
        if key not in ids:
            ids[key] = len(ids)
        group_of_pair[d] = ids[key]
    return group_of_pair, len(ids)


def select_groups(group_scene: np.ndarray, seed: int, step: int, budget: int) -> np.ndarray:
    """Boolean mask over groups: per scene, the min(|E_scene|, budget) groups
    with the smallest (key, group)."""
    group_scene = np.asarray(group_scene, np.int64)
    sel = np.zeros(group_scene.size, bool)
    for s in np.unique(group_scene):
        gs = np.flatnonzero(group_scene == s)
        keyed = sorted((group_key(seed, step, int(g)), int(g)) for g in gs)
        for _, g in keyed[:min(len(gs), budget)]:
            sel[g] = True
    return sel


def selected_pairs(pairs: np.ndarray, scene_of_pair: np.ndarray, seed: int, step: int,
                   budget: int) -> np.ndarray:
    """Boolean mask over directed pairs selected at `step`."""
    group_of_pair, n_groups = pair_groups(pairs)
    group_scene = np.zeros(n_groups, np.int64)
    group_scene[group_of_pair] = np.asarray(scene_of_pair, np.int64)
    return select_groups(group_scene, seed, step, budget)[group_of_pair]
