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
same bits as a serial evaluation).  <name>_envelope.npz holds the oracle's
own sensitivity over those prefixes: the same runs with every gradient
perturbed by a seeded random relative amount (1e-9, 5e-8), and how far each
ends from the stored prefix; <name>_window_envelope.npz the same for each
10-step window of a whole run (c2), restarted from the stored states;
<name>_run_envelope.npz the same for the whole run (c2) from the initial
poses.
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


# oracle self-sensitivity: the prefix runs again with every gradient moved by
# a seeded random perturbation of relative (normwise) size eps
ENVELOPE = {"c3": ((1e-9, 5e-8), (0, 1, 2)), "c5": ((1e-9, 5e-8), (0, 1, 2)),
            "c4": ((1e-9, 5e-8), (0,))}


def rotation_deg(a, b):
    c = np.clip((np.trace(a @ b.T) - 1.0) / 2.0, -1.0, 1.0)
    return float(np.degrees(np.arccos(c)))


def write_envelope(name: str, workers=None):
    """How far the oracle's own trajectory moves when its gradients are
    perturbed at the level of rounding differences: per run (eps, seed), the
    loss's relative deviation at every step and the largest rotation and
    camera-centre deviation over the views at every stored snapshot, against
    the stored prefix."""
    import time
    g = np.load(os.path.join(HERE, f"{name}_prefix.npz"), allow_pickle=False)
    n = int(g["iterations"])
    prob = make(name)
    assert str(g["checksum"]) == input_checksum(prob)
    d2 = opar.distance_fields(prob, workers)
    op = ocost.OracleProblem(prob, d2=d2)
    del d2
    epss, seeds = ENVELOPE[name]
    runs, loss_dev, rot_dev, ctr_dev = [], [], [], []
    with opar.ParallelEvaluator(op, workers, single_threaded=True) as ev:
        for eps in epss:
            for seed in seeds:
                t0 = time.time()
                rng = np.random.default_rng([seed, 7])

                def evaluate(poses, lam, params, selected=None, eps=eps, rng=rng):
                    r = ev(poses, lam, params, selected=selected)
                    e = rng.normal(size=r["grad"].shape)
                    r["grad"] = r["grad"] + eps * np.linalg.norm(r["grad"]) / np.linalg.norm(e) * e
                    return r

                hist = oloop.run(op, prob.poses_init, n, record_every=1, evaluate=evaluate)
                loss = np.array(hist["loss"])
                loss_dev.append((np.abs(loss - g["loss"]) / np.abs(g["loss"])).max(axis=1))
                rots, ctrs = [], []
                for k, st in enumerate(g["steps_at"]):
                    P = hist["poses"][int(st)] if st < n else hist["final_poses"]
                    Q = g["poses_at"][k]
                    rots.append(max(rotation_deg(P[v][:, :3], Q[v][:, :3]) for v in range(len(P))))
                    cp = -np.einsum("vji,vj->vi", P[:, :, :3], P[:, :, 3])
                    cq = -np.einsum("vji,vj->vi", Q[:, :, :3], Q[:, :, 3])
                    ctrs.append(float(np.linalg.norm(cp - cq, axis=1).max()))
                rot_dev.append(rots)
                ctr_dev.append(ctrs)
                runs.append((eps, seed))
                print(f"{name}: eps {eps:.0e} seed {seed}: rotation deviation by snapshot "
                      + ", ".join(f"{a:.2e}" for a in rots) + f" deg ({time.time() - t0:.0f} s)",
                      flush=True)
    np.savez_compressed(
        os.path.join(HERE, f"{name}_envelope.npz"), eps=np.array([r[0] for r in runs]),
        seed=np.array([r[1] for r in runs]), loss_dev=np.array(loss_dev),
        rot_dev=np.array(rot_dev), ctr_dev=np.array(ctr_dev), steps_at=g["steps_at"],
        checksum=g["checksum"])


def write_window_envelope(name: str, workers=None, epss=(1e-9, 5e-8), seeds=(0, 1, 2)):
    """The oracle's own sensitivity over the 10-step windows of a whole run:
    each window restarted from the stored state (poses, Adam moments, step)
    with every gradient perturbed by a seeded random relative amount, and how
    far it ends from the stored state of the next window (largest rotation
    and camera-centre deviation over the views) and how far its losses are
    from the stored ones."""
    import time
    g = np.load(os.path.join(HERE, f"{name}_trajectory.npz"), allow_pickle=False)
    n = int(g["iterations"])
    prob = make(name)
    assert str(g["checksum"]) == input_checksum(prob)
    op = ocost.OracleProblem(prob)
    n_win = g["poses_every10"].shape[0] - 1
    runs, loss_dev, rot_dev = [], [], []
    with opar.ParallelEvaluator(op, workers, single_threaded=True) as ev:
        for eps in epss:
            for seed in seeds:
                t0 = time.time()
                rng = np.random.default_rng([seed, 11])

                def evaluate(poses, lam, params, selected=None, eps=eps, rng=rng):
                    r = ev(poses, lam, params, selected=selected)
                    e = rng.normal(size=r["grad"].shape)
                    r["grad"] = r["grad"] + eps * np.linalg.norm(r["grad"]) / np.linalg.norm(e) * e
                    return r

                ld, rd = [], []
                for k in range(n_win):
                    steps = min(10, n - 10 * k)
                    hist = oloop.run(op, g["poses_every10"][k], steps, start_step=10 * k,
                                     m0=g["m_every10"][k], v0=g["v_every10"][k], evaluate=evaluate)
                    loss = np.array(hist["loss"])[:, 0]
                    ref = g["loss"][10 * k:10 * k + steps, 0]
                    ld.append(float((np.abs(loss - ref) / np.abs(ref)).max()))
                    P, Q = hist["final_poses"], g["poses_every10"][k + 1]
                    rd.append(max(rotation_deg(P[v][:, :3], Q[v][:, :3]) for v in range(len(P))))
                loss_dev.append(ld)
                rot_dev.append(rd)
                runs.append((eps, seed))
                print(f"{name} windows: eps {eps:.0e} seed {seed}: worst window rotation "
                      f"{max(rd):.2e} deg, loss {max(ld):.2e} ({time.time() - t0:.0f} s)", flush=True)
    np.savez_compressed(
        os.path.join(HERE, f"{name}_window_envelope.npz"), eps=np.array([r[0] for r in runs]),
        seed=np.array([r[1] for r in runs]), loss_dev=np.array(loss_dev),
        rot_dev=np.array(rot_dev), checksum=g["checksum"])


def write_run_envelope(name: str, workers=None, epss=(1e-9, 5e-8), seeds=(0, 1, 2)):
    """The oracle's own sensitivity over a whole stored run (c2): the run
    repeated from the initial poses with every gradient perturbed by a seeded
    random relative amount, and how far it is from the stored run every 10
    steps (largest rotation deviation over the views) and at every step in
    loss."""
    import time
    g = np.load(os.path.join(HERE, f"{name}_trajectory.npz"), allow_pickle=False)
    n = int(g["iterations"])
    prob = make(name)
    assert str(g["checksum"]) == input_checksum(prob)
    op = ocost.OracleProblem(prob)
    runs, loss_dev, rot_dev = [], [], []
    with opar.ParallelEvaluator(op, workers, single_threaded=True) as ev:
        for eps in epss:
            for seed in seeds:
                t0 = time.time()
                rng = np.random.default_rng([seed, 13])

                def evaluate(poses, lam, params, selected=None, eps=eps, rng=rng):
                    r = ev(poses, lam, params, selected=selected)
                    e = rng.normal(size=r["grad"].shape)
                    r["grad"] = r["grad"] + eps * np.linalg.norm(r["grad"]) / np.linalg.norm(e) * e
                    return r

                hist = oloop.run(op, prob.poses_init, n, record_every=1, evaluate=evaluate)
                loss = np.array(hist["loss"])[:, 0]
                loss_dev.append(np.abs(loss - g["loss"][:, 0]) / np.abs(g["loss"][:, 0]))
                snaps = [hist["poses"][10 * k] if 10 * k < n else hist["final_poses"]
                         for k in range(1, g["poses_every10"].shape[0])]
                rot_dev.append([max(rotation_deg(P[v][:, :3], Q[v][:, :3]) for v in range(len(P)))
                                for P, Q in zip(snaps, g["poses_every10"][1:])])
                runs.append((eps, seed))
                print(f"{name} run: eps {eps:.0e} seed {seed}: rotation deviation at the end "
                      f"{rot_dev[-1][-1]:.2e} deg ({time.time() - t0:.0f} s)", flush=True)
    np.savez_compressed(
        os.path.join(HERE, f"{name}_run_envelope.npz"), eps=np.array([r[0] for r in runs]),
        seed=np.array([r[1] for r in runs]), loss_dev=np.array(loss_dev),
        rot_dev=np.array(rot_dev), checksum=g["checksum"])


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(ITERS) + list(PREFIX) + [k + "_envelope" for k in ENVELOPE]):
        if name.endswith("_run_envelope"):
            write_run_envelope(name[:-len("_run_envelope")])
        elif name.endswith("_window_envelope"):
            write_window_envelope(name[:-len("_window_envelope")])
        elif name.endswith("_envelope"):
            write_envelope(name[:-len("_envelope")])
        elif name in PREFIX:
            write_prefix(name)
        else:
            write(name)
