"""Oracle: the same evaluation spread over worker processes.

Test infrastructure only (see the package header).

Nothing of the method is computed here.  The distance transforms of the
views and the per-pair sums of OracleProblem.direction are computed in forked
worker processes (which share the problem's arrays), and
OracleProblem.evaluate combines the per-pair sums in pair order exactly as
it does serially, so the loss and gradients are the same bits as a serial
evaluation (tested).  Used to write stored trajectories of the larger
workloads and to time the oracle on every host core.
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

from . import edt as _edt
from .cost import CostParams, OracleProblem

_STATE = {}
_KEYS = ("S", "n", "n_src", "G_tgt", "G_src", "F_tgt", "F_src")


def _edt_work(args):
    v, edge = args
    return v, _edt.edt_separable(edge).astype(np.int32)


def _pair_work(args):
    ids, poses, lam, params = args
    op = _STATE["op"]
    out = {}
    for d in ids:
        r = op.direction(int(d), poses, float(lam[int(op.scene_of_pair[d])]), params)
        out[int(d)] = {k: r[k] for k in _KEYS}
    return out


def _single_threaded():
    """Worker initializer: one BLAS thread per worker process, so that the
    workers are the only parallelism (for timing)."""
    from threadpoolctl import threadpool_limits
    _STATE["limits"] = threadpool_limits(1)


def default_workers() -> int:
    return max(1, min(os.cpu_count() or 1, 16))


def distance_fields(prob, workers: int | None = None, views=None, context: str = "fork"):
    """{view: exact d2} of the oracle's own transform, views spread over
    workers.  The edge maps go to the workers as arguments, so `context` may
    be "spawn" (fresh interpreters, for a parent that holds a GPU context)."""
    views = list(range(prob.n_views)) if views is None else list(views)
    jobs = ((v, prob.edge_map(v)) for v in views)
    with mp.get_context(context).Pool(workers or default_workers(),
                                      initializer=_single_threaded) as pool:
        out = dict(pool.imap_unordered(_edt_work, jobs, chunksize=1))
    return out


class ParallelEvaluator:
    """op.evaluate(poses, lam, params, selected=None) over `workers`
    processes; pairs are dealt to chunks of about equal residual counts.
    `pair_ids` restricts the evaluation to those directed pairs (the problem
    then needs only their views); `single_threaded` limits each worker to one
    BLAS thread."""

    def __init__(self, op: OracleProblem, workers: int | None = None, chunks_per_worker=4,
                 pair_ids=None, single_threaded=False):
        self.op = op
        self.workers = workers or default_workers()
        self.pair_ids = None if pair_ids is None else [int(d) for d in pair_ids]
        _STATE["op"] = op
        self.pool = mp.get_context("fork").Pool(
            self.workers, initializer=_single_threaded if single_threaded else None)
        ids = np.arange(op.pairs.shape[0]) if pair_ids is None else np.asarray(self.pair_ids)
        cost = np.zeros(op.pairs.shape[0])
        cost[ids] = [op.pts[int(op.pairs[d, 0])][0].size for d in ids]
        order = ids[np.argsort(-cost[ids], kind="stable")]
        n_chunks = max(1, min(len(order), self.workers * chunks_per_worker))
        load = np.zeros(n_chunks)
        self.chunks = [[] for _ in range(n_chunks)]
        for d in order:                          # longest first onto the lightest chunk
            k = int(np.argmin(load))
            self.chunks[k].append(int(d))
            load[k] += cost[d]
        self.chunks = [c for c in self.chunks if c]

    def close(self):
        self.pool.close()
        self.pool.join()
        _STATE.pop("op", None)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __call__(self, poses, lam, params: CostParams = CostParams(), selected=None):
        lam = np.broadcast_to(np.asarray(lam, np.float64), (self.op.n_scenes,)).copy()
        jobs = []
        for c in self.chunks:
            ids = c if selected is None else [d for d in c if selected[d]]
            if ids:
                jobs.append((ids, poses, lam, params))
        res = {}
        for part in self.pool.imap_unordered(_pair_work, jobs):
            res.update(part)
        return self.op.evaluate(poses, lam, params, selected=selected, pair_results=res,
                                pair_ids=self.pair_ids)
