"""GPU: whole optimisation runs (captured iteration and eager calls) against
the oracle's trajectories, and the pose step against the oracle's Adam step."""
import os

import numpy as np
import pytest
import torch

from oracle import loop as oloop
from tests.gpu_helpers import problem, rel_norm_err, rotation_angle_deg, say

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    from tests.golden.make_golden import input_checksum
    g = np.load(os.path.join(GOLDEN, f"{name}_trajectory.npz"), allow_pickle=False)
    assert str(g["checksum"]) == input_checksum(problem(name)), "generator changed: rerun make_golden"
    return g


def run_captured(prob, n, snapshot_every=None):
    """The captured iteration run n steps from the initial poses: the loss
    of every step and the final poses (and, with snapshot_every, the poses
    after every that many steps)."""
    from paper_2607_00579_amd.api import EdgePlan
    dev = torch.device("cuda:0")
    plan = EdgePlan.from_problem(prob, device=dev)
    poses = torch.from_numpy(prob.poses_init.copy()).to(dev)
    m = torch.zeros(prob.n_views, 6, dtype=torch.float64, device=dev)
    v = torch.zeros_like(m)
    step = torch.zeros(1, dtype=torch.int32, device=dev)
    loss = torch.zeros(plan.n_scenes, dtype=torch.float64, device=dev)
    plan.capture_iteration(poses, m, v, step, loss)
    hist = torch.zeros(n, plan.n_scenes, dtype=torch.float64, device=dev)
    snaps = []
    for s in range(n):
        plan.launch_iteration()
        hist[s] = loss
        if snapshot_every and (s + 1) % snapshot_every == 0:
            snaps.append(poses.clone())
    torch.cuda.synchronize()
    assert int(step.item()) == n
    if snapshot_every:
        return hist.cpu().numpy(), poses.cpu().numpy(), [q.cpu().numpy() for q in snaps]
    return hist.cpu().numpy(), poses.cpu().numpy()


def run_eager(prob, n):
    from paper_2607_00579_amd import _lib
    from paper_2607_00579_amd.api import EdgePlan
    dev = torch.device("cuda:0")
    plan = EdgePlan.from_problem(prob, device=dev)
    poses = torch.from_numpy(prob.poses_init.copy()).to(dev)
    m = torch.zeros(prob.n_views, 6, dtype=torch.float64, device=dev)
    v = torch.zeros_like(m)
    step = torch.zeros(1, dtype=torch.int32, device=dev)
    lam = torch.zeros(plan.n_scenes, dtype=torch.float32, device=dev)
    lr = torch.zeros(plan.n_scenes, dtype=torch.float64, device=dev)
    hist = []
    st = torch.cuda.current_stream().cuda_stream
    for s in range(n):
        _lib.schedule(step, plan.n_scenes, 10.0, 6.0, 1000, 3e-3, 25, 2000, lam, lr, st)
        o = plan.cost(poses, lam, grad=True)
        hist.append(o["loss"].clone())
        plan.pose_step(poses, m, v, o["grad"], lr, step)
    torch.cuda.synchronize()
    return torch.stack(hist).cpu().numpy(), poses.cpu().numpy()


def pose_diffs(a, b):
    ang = max(rotation_angle_deg(a[k][:, :3], b[k][:, :3]) for k in range(a.shape[0]))
    ca = -np.einsum("vji,vj->vi", a[:, :, :3], a[:, :, 3])
    cb = -np.einsum("vji,vj->vi", b[:, :, :3], b[:, :, 3])
    return ang, float(np.linalg.norm(ca - cb, axis=1).max())


def compare(name, hist, final, g, rot_tol):
    ref_loss = g["loss"]
    n = int(g["iterations"])
    rel = np.abs(hist[:, 0] - ref_loss[:, 0]) / np.abs(ref_loss[:, 0])
    ang, dc = pose_diffs(final, g["final_poses"])
    say(f"{name}: {n} iters, loss rel err first 10 {rel[:10].max():.2e}, all {rel.max():.2e}, "
        f"final rotation diff max {ang:.2e} deg, centre diff {dc:.2e}")
    assert rel[:10].max() < 1e-5
    assert ang < rot_tol


def test_captured_iteration_trajectory_c1(gpu):
    """50 steps: the whole run stays within 0.01 deg of the oracle."""
    g = golden("c1")
    hist, final = run_captured(problem("c1"), int(g["iterations"]))
    compare("c1 graph", hist, final, g, rot_tol=0.01)


def test_captured_iteration_trajectory_c2_full_run(gpu):
    """200 steps from the initial poses.  The run is chaotic: the oracle
    against itself with its gradients perturbed by 1e-9 or 5e-8 relative
    (three seeds each, c2_run_envelope.npz) stays within 1e-5 deg for about
    30 steps, then the gap grows about 30x per 10 steps and saturates near
    0.05 deg.  The GPU's poses every 10 steps are held to max(0.01 deg, 3x
    the oracle's own spread so far), its first 10 losses to 1e-5; the 10-step
    windows below carry the tighter bar."""
    g = golden("c2")
    n = int(g["iterations"])
    hist, final, snaps = run_captured(problem("c2"), n, snapshot_every=10)
    compare("c2 graph", hist, final, g, rot_tol=0.2)
    from tests.golden.make_golden import input_checksum
    env = np.load(os.path.join(GOLDEN, "c2_run_envelope.npz"), allow_pickle=False)
    assert str(env["checksum"]) == input_checksum(problem("c2")), "generator changed: rerun make_golden"
    rot = np.array([pose_diffs(P, Q)[0] for P, Q in zip(snaps, g["poses_every10"][1:])])
    env_rot = np.maximum.accumulate(env["rot_dev"].max(axis=0))
    bar = np.maximum(ROT_BAR, ENVELOPE_FACTOR * env_rot)
    k = int(np.argmax(rot / bar))
    say(f"c2 run: rotation diff every 10 steps up to {rot.max():.2e} deg; worst against its bar "
        f"{rot[k]:.2e} of {bar[k]:.2e} at step {10 * (k + 1)} (oracle's own {env_rot[k]:.2e})")
    assert (rot <= bar).all(), (rot, bar)


# The oracle's own spread at step s: the largest deviation from the stored
# trajectory that any of its perturbed runs (gradients moved by 1e-9 and 5e-8
# relative, several seeds) shows at or before s.  The GPU's poses may deviate
# by ENVELOPE_FACTOR times that spread, never less than the spec bar;
# its losses are held to LOSS_BAR while the oracle's own loss spread stays
# below LOSS_BAR / ENVELOPE_FACTOR, and afterwards, when the poses carry the
# comparison, to LOSS_SANITY times the spread (a handful of sampled runs
# underestimate the tail of a chaotic spread: on the 32-view workload the
# GPU's loss leads the sampled spread by up to 3.5x around steps 12-15 while
# its rotations stay inside it).
ENVELOPE_FACTOR = 3.0
LOSS_SANITY = 10.0
ROT_BAR = 0.01          # degrees
LOSS_BAR = 1e-5         # relative

WINDOW_BAR = 1e-3      # degrees, at the end of a 10-step window


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_trajectory_windows_from_oracle_states(gpu, name):
    """Restart the captured iteration from the oracle's state (poses, Adam
    moments, step) every 10 steps and run 10 steps.  Every window must end
    within 1e-3 deg of the oracle and every loss within 1e-5, or, where the
    oracle itself is that sensitive, within three times the spread the
    oracle shows over the same window when its gradients are perturbed at
    rounding size (1e-9 and 5e-8 relative, three seeds each; stored with the
    whole run in <name>_window_envelope.npz)."""
    from paper_2607_00579_amd.api import EdgePlan
    g = golden(name)
    prob = problem(name)
    dev = torch.device("cuda:0")
    plan = EdgePlan.from_problem(prob, device=dev)
    poses = torch.zeros(prob.n_views, 3, 4, dtype=torch.float64, device=dev)
    m = torch.zeros(prob.n_views, 6, dtype=torch.float64, device=dev)
    v = torch.zeros_like(m)
    step = torch.zeros(1, dtype=torch.int32, device=dev)
    loss = torch.zeros(plan.n_scenes, dtype=torch.float64, device=dev)
    plan.capture_iteration(poses, m, v, step, loss)
    n_win = g["poses_every10"].shape[0] - 1
    ang = np.zeros(n_win)
    lerr = np.zeros(n_win)
    for k in range(n_win):
        poses.copy_(torch.from_numpy(g["poses_every10"][k]))
        m.copy_(torch.from_numpy(g["m_every10"][k]))
        v.copy_(torch.from_numpy(g["v_every10"][k]))
        step.fill_(10 * k)
        steps = min(10, int(g["iterations"]) - 10 * k)
        for s in range(steps):
            plan.launch_iteration()
            ref = g["loss"][10 * k + s, 0]
            lerr[k] = max(lerr[k], abs(float(loss[0].item()) - ref) / abs(ref))
        ang[k] = pose_diffs(poses.cpu().numpy(), g["poses_every10"][k + 1])[0]
    bar_rot = np.full(n_win, WINDOW_BAR)
    bar_loss = np.full(n_win, LOSS_BAR)
    path = os.path.join(GOLDEN, f"{name}_window_envelope.npz")
    if os.path.exists(path):
        from tests.golden.make_golden import input_checksum
        env = np.load(path, allow_pickle=False)
        assert str(env["checksum"]) == input_checksum(prob), "generator changed: rerun make_golden"
        env_rot, env_loss = env["rot_dev"].max(axis=0), env["loss_dev"].max(axis=0)
        bar_rot = np.maximum(bar_rot, ENVELOPE_FACTOR * env_rot)
        bar_loss = np.maximum(bar_loss, ENVELOPE_FACTOR * env_loss)
        say(f"{name}: oracle's own window spread up to {env_rot.max():.2e} deg, "
            f"{int((ENVELOPE_FACTOR * env_rot > WINDOW_BAR).sum())} of {n_win} windows above "
            f"a third of the bar")
    else:
        assert name == "c1", f"{path} missing: run tests/golden/make_golden.py"
    k = int(np.argmax(ang / bar_rot))
    say(f"{name}: {n_win} windows of 10 steps: worst rotation diff {ang.max():.2e} deg, "
        f"worst against its bar {ang[k]:.2e} of {bar_rot[k]:.2e} (window {k}); "
        f"worst loss rel err {lerr.max():.2e}")
    assert (ang <= bar_rot).all(), (ang, bar_rot)
    assert (lerr <= bar_loss).all(), (lerr, bar_loss)


def golden_prefix(name):
    from tests.golden.make_golden import input_checksum
    g = np.load(os.path.join(GOLDEN, f"{name}_prefix.npz"), allow_pickle=False)
    assert str(g["checksum"]) == input_checksum(problem(name)), "generator changed: rerun make_golden"
    return g


def golden_envelope(name):
    from tests.golden.make_golden import input_checksum
    e = np.load(os.path.join(GOLDEN, f"{name}_envelope.npz"), allow_pickle=False)
    assert str(e["checksum"]) == input_checksum(problem(name)), "generator changed: rerun make_golden"
    return e




@pytest.mark.parametrize("name", ["c3", "c5", "c4"])
def test_trajectory_prefix_from_initial_poses(gpu, name):
    """The captured iteration from the initial poses, in the benchmark's
    launch configuration (autotuned schedule), against the oracle's first 20
    (c3, c5) or 10 (c4, all 64 scenes) steps.  Every pose is held to 0.01 deg
    of rotation and every scene's loss to 1e-5 relative for as long as the
    oracle itself stays that close to its own trajectory under rounding-size
    perturbations of its gradients; past that point (the cost is piecewise
    bilinear with about a million cell-boundary kinks, and Adam's normalised
    steps pass small gradient differences on at full size, so rounding
    differences grow by orders of magnitude within a few steps) the poses are
    held to three times the oracle's own spread, stored with the prefix."""
    from paper_2607_00579_amd.api import EdgePlan
    g = golden_prefix(name)
    env = golden_envelope(name)
    prob = problem(name)
    n = int(g["iterations"])
    dev = torch.device("cuda:0")
    plan = EdgePlan.from_problem(prob, device=dev)
    poses = torch.from_numpy(prob.poses_init.copy()).to(dev)
    chosen = plan.autotune(poses, 10.0, iters=1)
    m = torch.zeros(prob.n_views, 6, dtype=torch.float64, device=dev)
    v = torch.zeros_like(m)
    step = torch.zeros(1, dtype=torch.int32, device=dev)
    loss = torch.zeros(plan.n_scenes, dtype=torch.float64, device=dev)
    plan.capture_iteration(poses, m, v, step, loss)
    hist = torch.zeros(n, plan.n_scenes, dtype=torch.float64, device=dev)
    snaps = {}
    at = set(int(k) for k in g["steps_at"])
    for s in range(n):
        plan.launch_iteration()
        hist[s] = loss
        if s + 1 in at:
            snaps[s + 1] = poses.clone()
    torch.cuda.synchronize()
    rel = (np.abs(hist.cpu().numpy() - g["loss"]) / np.abs(g["loss"])).max(axis=1)
    rot = np.array([pose_diffs(snaps[int(st)].cpu().numpy(), g["poses_at"][k])[0]
                    for k, st in enumerate(g["steps_at"])])
    env_rot = np.maximum.accumulate(env["rot_dev"].max(axis=0))
    env_loss = np.maximum.accumulate(env["loss_dev"].max(axis=0))
    bar_rot = np.maximum(ROT_BAR, ENVELOPE_FACTOR * env_rot)
    chaotic = ENVELOPE_FACTOR * env_loss >= LOSS_BAR
    bar_loss = np.where(chaotic, np.maximum(LOSS_BAR, LOSS_SANITY * env_loss), LOSS_BAR)
    say(f"{name} prefix ({plan.n_residuals} residuals/step, schedule {chosen}): {n} steps; "
        + "rotation diff by step " + ", ".join(
            f"{int(st)}: {a:.2e} (oracle's own {e:.2e})"
            for st, a, e in zip(g["steps_at"], rot, env_rot))
        + f" deg; loss rel err {rel.max():.2e} (oracle's own up to {env_loss.max():.2e})")
    assert (rot <= bar_rot).all(), (rot, bar_rot)
    assert (rel <= bar_loss).all(), (rel, bar_loss)
    # where the first snapshot lies before the oracle's own spread reaches
    # the bar, the GPU is held to the bar itself there (on the 64-scene batch
    # the oracle's spread passes it within five steps)
    if env_rot[0] < ROT_BAR / ENVELOPE_FACTOR:
        assert rot[0] < ROT_BAR
    assert plan.device_status() == 0


def test_eager_trajectory_c1_equals_captured(gpu):
    g = golden("c1")
    n = int(g["iterations"])
    h1, f1 = run_eager(problem("c1"), n)
    h2, f2 = run_captured(problem("c1"), n)
    compare("c1 eager", h1, f1, g, rot_tol=0.01)
    assert np.array_equal(h1, h2) and np.array_equal(f1, f2)


def test_pose_step_matches_oracle(gpu):
    from paper_2607_00579_amd import _lib
    rng = np.random.default_rng(7)
    V = 37
    poses = np.stack([np.concatenate([np.linalg.qr(rng.normal(size=(3, 3)))[0] * 1.0,
                                      rng.normal(size=(3, 1)) * 3], 1) for _ in range(V)])
    for k in range(V):
        if np.linalg.det(poses[k, :, :3]) < 0:
            poses[k, :, :3] *= -1
    dev = torch.device("cuda:0")
    P = torch.from_numpy(poses.copy()).to(dev)
    m = torch.zeros(V, 6, dtype=torch.float64, device=dev)
    v = torch.zeros_like(m)
    step = torch.zeros(1, dtype=torch.int32, device=dev)
    fixed = torch.from_numpy((np.arange(V) % 5 == 0).astype(np.uint8)).to(dev)
    sov = torch.from_numpy((np.arange(V) % 3).astype(np.int32)).to(dev)
    lrs = np.array([1e-2, 3e-3, 0.5])
    lr = torch.from_numpy(lrs).to(dev)
    ref_p, ref_m, ref_v = poses.copy(), np.zeros((V, 6)), np.zeros((V, 6))
    st = torch.cuda.current_stream().cuda_stream
    for s in range(1, 6):
        g = rng.normal(size=(V, 6)) * 10 ** rng.uniform(-3, 2, size=(V, 1))
        G = torch.from_numpy(g).to(dev)
        _lib.pose_step(P, m, v, G, V, sov, fixed, lr, 0.9, 0.999, 1e-8, step, st)
        ref_p, ref_m, ref_v = oloop.adam_se3_step(ref_p, ref_m, ref_v, g, s, lrs,
                                                  fixed=(np.arange(V) % 5 == 0),
                                                  scene_of_view=np.arange(V) % 3)
    torch.cuda.synchronize()
    assert int(step.item()) == 5
    assert np.abs(P.cpu().numpy() - ref_p).max() < 1e-12
    assert np.abs(m.cpu().numpy() - ref_m).max() < 1e-12
    assert rel_norm_err(v.cpu().numpy(), ref_v) < 1e-12


def test_schedule_matches_oracle(gpu):
    from paper_2607_00579_amd import _lib
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream().cuda_stream
    for s in (0, 1, 24, 25, 26, 500, 999, 1000, 1500, 1999):
        step = torch.tensor([s], dtype=torch.int32, device=dev)
        lam = torch.zeros(3, dtype=torch.float32, device=dev)
        lr = torch.zeros(3, dtype=torch.float64, device=dev)
        _lib.schedule(step, 3, 10.0, 6.0, 1000, 3e-3, 25, 2000, lam, lr, st)
        torch.cuda.synchronize()
        assert np.allclose(lam.cpu().numpy(), oloop.clamp_lambda(s), rtol=1e-6)
        assert np.allclose(lr.cpu().numpy(), oloop.learning_rate(s), rtol=1e-12)
