"""The process-parallel oracle evaluation (used for the stored prefix
trajectories and the host-core timing) gives the same bits as the serial
oracle: distance transforms, loss, gradients and a three-step loop."""
import numpy as np

from oracle import cost, loop, parallel
from synth import make


def test_parallel_evaluation_is_bitwise_serial():
    p = make("c2")
    op = cost.OracleProblem(p)
    d2 = parallel.distance_fields(p, 3)
    assert all(np.array_equal(d2[v], op.d2[v]) for v in range(p.n_views))
    want = op.evaluate(p.poses_init, 8.0)
    with parallel.ParallelEvaluator(op, 3, single_threaded=True) as ev:
        got = ev(p.poses_init, 8.0)
        for k in ("loss", "grad", "grad_focal", "S", "n", "L", "w", "G_tgt", "G_src"):
            assert np.array_equal(got[k], want[k]), k
        h1 = loop.run(op, p.poses_init, 3)
        h2 = loop.run(op, p.poses_init, 3, evaluate=ev)
    assert np.array_equal(h1["final_poses"], h2["final_poses"])
    assert np.array_equal(np.array(h1["loss"]), np.array(h2["loss"]))


def test_parallel_evaluation_of_a_pair_subset():
    """Restricted to some pairs (the problem holding only their views): the
    same bits as the serial evaluation of those pairs."""
    p = make("c2")
    ids = [d for d in range(p.n_pairs) if p.pairs[d, 0] < 4 and p.pairs[d, 1] < 4]
    op = cost.OracleProblem(p, views=range(4))
    want = op.evaluate(p.poses_init, 10.0, pair_ids=ids)
    with parallel.ParallelEvaluator(op, 2, pair_ids=ids, single_threaded=True) as ev:
        got = ev(p.poses_init, 10.0)
    assert np.array_equal(got["loss"], want["loss"]) and np.array_equal(got["grad"], want["grad"])
