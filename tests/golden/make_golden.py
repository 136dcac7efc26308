"""Write the oracle trajectories the GPU trajectory tests compare against.

    python tests/golden/make_golden.py [c1 c2 c3 c4 c5 ...]

Calls only the FP64 oracle (oracle/) and the seeded input generator (synth/).
Each file stores, for one workload, the oracle's loss and gradient norm at every
iteration, the poses (and, for the whole runs of c1 and c2, the Adam moments)
at regular steps and at the end, and a checksum of the generated inputs so
that a generator change is detected instead of silently comparing against
stale values.  c1 and c2 are whole runs (c1_trajectory.npz, c2_trajectory.npz);
c3, c4 and c5 are prefixes of their runs (20, 10 and 20 steps,
<name>_prefix.npz), evaluated over worker processes (oracle.parallel; the
same bits as a serial evaluation).
"""
from __future__ import annotations

import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import cost as ocost  # noqa: E402
from oracle import loop as oloop  # noqa: E402
from oracle import parallel as opar  # noqa: E402
from synth import make  # noqa: E402

ITERS = {"c1": 50, "c2": 200}
PREFIX = {"c3": (20, 5), "c5": (20, 5), "c4": (10, 5)}    # steps, pose snapshot interval


def input_checksum(prob) -> str:
    h = hashlib.sha256()
    for a in (prob.edge_flat, prob.depth_flat, prob.poses_init, prob.pairs, prob.K):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def write(name: str):
    prob = make(name)
    op = ocost.OracleProblem(prob)
    n = ITERS[name]
    hist = oloop.run(op, prob.poses_init, n, record_every=1)
    # the state each 10-step window starts from (poses, Adam moments), plus
    # the end state
    poses10 = np.stack(hist["poses"][::10] + [hist["final_poses"]])
    m10 = np.stack(hist["m_hist"][::10] + [hist["m"]])
    v10 = np.stack(hist["v_hist"][::10] + [hist["v"]])
    np.savez_compressed(
        os.path.join(HERE, f"{name}_trajectory.npz"),
        loss=np.array(hist["loss"]), grad_norm=np.array(hist["grad_norm"]),
        poses_every10=poses10, m_every10=m10, v_every10=v10, final_poses=hist["final_poses"],
        checksum=np.array(input_checksum(prob)), iterations=np.array(n))
    print(f"{name}: {n} iterations, loss {hist['loss'][0][0]:.6f} -> {hist['loss'][-1][0]:.6f}")


def write_prefix(name: str, workers=None):
    import time
    n, every = PREFIX[name]
    t0 = time.time()
    prob = make(name)
    print(f"{name}: generated in {time.time() - t0:.0f} s", flush=True)
    t0 = time.time()
    d2 = opar.distance_fields(prob, workers)
    op = ocost.OracleProblem(prob, d2=d2)
    del d2
    print(f"{name}: distance transforms in {time.time() - t0:.0f} s", flush=True)
    t0 = time.time()
    with opar.ParallelEvaluator(op, workers, single_threaded=True) as ev:
        hist = oloop.run(op, prob.poses_init, n, record_every=1, evaluate=ev)
    print(f"{name}: {n} steps in {time.time() - t0:.0f} s", flush=True)
    steps_at = np.arange(every, n + 1, every)
    poses_at = np.stack([hist["poses"][k] if k < n else hist["final_poses"] for k in steps_at])
    np.savez_compressed(
        os.path.join(HERE, f"{name}_prefix.npz"),
        loss=np.array(hist["loss"]), grad_norm=np.array(hist["grad_norm"]),
        steps_at=steps_at, poses_at=poses_at, checksum=np.array(input_checksum(prob)),
        iterations=np.array(n))
    print(f"{name}: loss {hist['loss'][0].sum():.6f} -> {hist['loss'][-1].sum():.6f}")


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(ITERS) + list(PREFIX)):
        if name in PREFIX:
            write_prefix(name)
        else:
            write(name)
