"""Write the oracle trajectories the GPU trajectory tests compare against.

    python tests/golden/make_golden.py [c1 c2 ...]

Calls only the FP64 oracle (oracle/) and the seeded input generator (synth/).
Each file stores, for one workload, the oracle's loss and gradient norm at every
iteration, the poses every 10 iterations and at the end, and a checksum of the
generated inputs so that a generator change is detected instead of silently
comparing against stale values.
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
from synth import make  # noqa: E402

ITERS = {"c1": 50, "c2": 200}


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


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(ITERS)):
        write(name)
