"""Trains the pose-proposal network on submap pairs that the mapping
pipeline itself generates, then stores the weights with the fallback cost
threshold.

Scenes: outdoor MAV-like workloads (120 x 80 m, 3000 frames, 0.1 m voxels,
30 submaps of 100 frames) for consecutive seeds.  Pairs: submaps i and j
(j = i+1..i+4) whose block overlap is at least 0.2, in both directions,
with the ground truth T_A_B from the generator's poses.  Training draws
re-framings of these pairs inside the library (covox_train_proposal: +-3 m
in x/y, +-0.5 m in z, +-180 deg yaw, +-2 deg roll/pitch of the prior).

Scenes stream through a window: each round maps --scenes-per-round new
scenes (the next one renders on the host while the GPU maps and trains),
drops the oldest beyond --window, and takes --steps-per-round Adam steps
on the pairs of the scenes in the window.  The learning rate falls in
steps (1, 1/3, 1/10 over the thirds of --total-steps, counted from
--step0), so that a run can continue an earlier one (--init, with the next
--seed0 and --step0).  The weights are stored after every round.

The fallback threshold (--calibrate) is the 95th percentile of the costs
that plain 8-start alignment reaches on the pairs it aligns successfully
(within 5 cm / 0.5 deg) in two calibration scenes (seeds 90 and up),
priors perturbed by +-0.5 m / +-10 deg yaw / +-2 deg roll and pitch.

Usage: python -m paper_2410_21149_amd.train_proposal [--rounds 5] [--out FILE]
Every step runs in the HIP library; this script only builds the inputs.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
DEFAULT_OUT = os.path.join(HERE, "data", "proposal_mav.npz")


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def block_pairs(ctx, subs, Tws, vs, min_overlap=0.2, reach=4):
    """(i, j, overlap) of submaps whose block-centre overlap is at least
    min_overlap: |A blocks containing T_gt B block centres| / min(|A|, |B|)."""
    keys = [ctx.export_blocks(s)["keys"] for s in subs]
    m = np.uint64(0x1FFFFF)
    coords = [np.stack([((k >> np.uint64(42)) & m).astype(np.int64), ((k >> np.uint64(21)) & m).astype(np.int64),
                        (k & m).astype(np.int64)], axis=-1) - (1 << 20) for k in keys]
    out = []
    for i in range(len(subs)):
        sa = set(map(tuple, coords[i]))
        for j in range(i + 1, min(len(subs), i + 1 + reach)):
            T = np.linalg.inv(Tws[i]) @ Tws[j]
            cb = (coords[j] + 0.5) * 8 * vs
            ia = np.floor((cb @ T[:3, :3].T + T[:3, 3]) / (8 * vs)).astype(np.int64)
            hit = sum(1 for t in map(tuple, ia) if t in sa)
            ov = hit / max(1, min(len(coords[i]), len(coords[j])))
            if ov >= min_overlap:
                out.append((i, j, ov))
    return out


def render_scene(seed, scale=1.0):
    """(workload, all frames) of one MAV scene, or None if the generator
    finds no path for this seed (host only)."""
    import scenegen as sg
    try:
        w = sg.mav(seed=seed, scale=scale)
    except RuntimeError:
        return None
    return w, w.frames()


def map_scene(cv, torch, ctx, w, frames):
    """Maps one rendered scene into gravity-aligned submaps of w.submap_every
    frames with current ESDFs (submaps that overflow the block capacity are
    skipped); returns (submaps, T_world_submap list)."""
    import scenegen as sg
    per = w.submap_every
    subs, Tws = [], []
    for k in range(w.n_frames // per):
        fr = torch.from_numpy(frames[k * per:(k + 1) * per]).cuda()
        T = sg.gravity_aligned(w.poses[k * per])
        s = ctx.submap_create(T)
        try:
            ctx.map_sequence(s, fr, w.cam.K, w.poses[k * per:(k + 1) * per], esdf_every=0)
        except cv.CovoxError:
            s.destroy()
            continue
        subs.append(s)
        Tws.append(T)
    ctx.update_esdf_batch(subs)
    return subs, Tws


def build_scene(cv, torch, ctx, seed, scale=1.0):
    """Renders and maps one MAV scene; returns (submaps, T_world_submap list)
    or None if the generator finds no path for this seed."""
    got = render_scene(seed, scale)
    if got is None:
        return None
    return map_scene(cv, torch, ctx, *got)


def scene_pairs(ctx, subs, Tws, vs=0.1, min_overlap=0.2):
    """Directed pairs (A, B, T_A_B) of one scene, both directions."""
    out = []
    for i, j, ov in block_pairs(ctx, subs, Tws, vs, min_overlap=min_overlap):
        T = np.linalg.inv(Tws[i]) @ Tws[j]
        out.append((subs[i], subs[j], T))
        out.append((subs[j], subs[i], np.linalg.inv(T)))
    return out


def perturbed(rng, T_gt, trans=0.5, yaw_deg=10.0, tilt_deg=2.0):
    c, s = math.cos, math.sin
    a = math.radians(rng.uniform(-yaw_deg, yaw_deg))
    b = math.radians(rng.uniform(-tilt_deg, tilt_deg))
    g = math.radians(rng.uniform(-tilt_deg, tilt_deg))
    Rz = np.array([[c(a), -s(a), 0], [s(a), c(a), 0], [0, 0, 1]])
    Ry = np.array([[c(b), 0, s(b)], [0, 1, 0], [-s(b), 0, c(b)]])
    Rx = np.array([[1, 0, 0], [0, c(g), -s(g)], [0, s(g), c(g)]])
    d = np.eye(4)
    d[:3, :3] = Rz @ Ry @ Rx
    d[:3, 3] = rng.uniform(-trans, trans, size=3)
    return T_gt @ d


def pose_error(T, G):
    dt = float(np.linalg.norm(T[:3, 3] - G[:3, 3]))
    cth = (np.trace(T[:3, :3] @ G[:3, :3].T) - 1) / 2
    return dt, math.degrees(math.acos(max(-1.0, min(1.0, cth))))


def lr_at(step, total, lr):
    """Step decay: lr, lr / 3, lr / 10 over the thirds of the total."""
    if step < total - 2 * (total // 3):
        return lr
    return lr / 3 if step < total - total // 3 else lr / 10


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--rounds", type=int, default=5)
    ap.add_argument("--scenes-per-round", type=int, default=20)
    ap.add_argument("--window", type=int, default=60, help="scenes kept on the device")
    ap.add_argument("--steps-per-round", type=int, default=1500)
    ap.add_argument("--total-steps", type=int, default=0, help="length of the learning-rate schedule (0: this run's)")
    ap.add_argument("--step0", type=int, default=0)
    ap.add_argument("--seed0", type=int, default=101)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--cell", type=float, default=1.0)
    ap.add_argument("--net-seed", type=int, default=1)
    ap.add_argument("--init", default=None, help="start from these stored weights (and their metadata)")
    ap.add_argument("--calibrate", action="store_true", help="compute the fallback threshold at the end")
    ap.add_argument("--block-capacity", type=int, default=8192, help="blocks per submap (submaps that overflow are skipped)")
    ap.add_argument("--render-scale", type=float, default=0.5,
                    help="render the training scenes at this fraction of 640x480 (same field of view)")
    ap.add_argument("--out", default=DEFAULT_OUT)
    a = ap.parse_args(argv)
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import concurrent.futures

    import torch

    import paper_2410_21149_amd as cv
    t0 = time.perf_counter()
    total = a.total_steps or a.rounds * a.steps_per_round
    meta = {"seeds": [], "pairs_train": 0, "steps": 0}
    ctx = cv.Context(voxel_size=0.1, trunc_vox=4, max_range=10.0, d_max=3.0, block_capacity=a.block_capacity)
    net = cv.Net(ctx, seed=a.net_seed)
    losses = []
    if a.init:
        params, meta0 = load(a.init)
        net.set_params(params)
        meta.update({k: meta0[k] for k in ("seeds", "pairs_train", "steps") if k in meta0})
        with np.load(a.init, allow_pickle=False) as z:
            losses = z["losses"].tolist()
    window = []  # (seed, submaps, pairs) of the scenes on the device
    pool = concurrent.futures.ThreadPoolExecutor(1)
    sd = a.seed0

    def next_render():
        nonlocal sd
        seed = sd
        sd += 1
        return seed, pool.submit(render_scene, seed, a.render_scale)

    pending = next_render()
    step = a.step0
    for r in range(a.rounds):
        added = 0
        # a continued run fills its window first, so that its first steps see as many pairs as later ones
        want = a.window if (a.init and r == 0) else a.scenes_per_round
        while added < want:
            seed, fut = pending
            pending = next_render()  # the next scene renders while this one maps
            got = fut.result()
            if got is None:
                continue
            subs, Tws = map_scene(cv, torch, ctx, *got)
            del got
            pairs = scene_pairs(ctx, subs, Tws)
            window.append((seed, subs, pairs))
            meta["seeds"].append(seed)
            meta["pairs_train"] += len(pairs)
            added += 1
            while len(window) > a.window:
                for s_ in window.pop(0)[1]:
                    s_.destroy()
        train = [p for _, _, ps in window for p in ps]
        _log("round %d: %d scenes in the window, %d pairs, %d distinct pairs so far (%.0f s)"
             % (r, len(window), len(train), meta["pairs_train"], time.perf_counter() - t0))
        left = a.steps_per_round
        while left > 0:
            m = min(250, left)
            lr = lr_at(step, a.step0 + total if a.total_steps == 0 else a.total_steps, a.lr)
            L = ctx.train_proposal(net, train, steps=m, batch=a.batch, lr=lr, cell=a.cell, seed=1000 + step)
            losses.extend(L.tolist())
            step += m
            left -= m
            _log("step %d lr %.2g loss %.4f (%.0f s)" % (step, lr, float(np.mean(L[-50:])), time.perf_counter() - t0))
        meta["steps"] = step
        save(a.out, net, losses, meta, a)
    pool.shutdown(wait=False, cancel_futures=True)
    for _, subs, _ in window:
        for s_ in subs:
            s_.destroy()
    if a.calibrate:
        # fallback threshold from plain 8-start on two calibration scenes
        cal, c_seeds, cs = [], [], 90
        while len(c_seeds) < 2:
            got = build_scene(cv, torch, ctx, cs, a.render_scale)
            if got is not None:
                cal += scene_pairs(ctx, *got)
                c_seeds.append(cs)
            cs += 1
        rng = np.random.default_rng(7)
        items = [(A, B, perturbed(rng, T)) for A, B, T in cal for _ in range(4)]
        Tq, cq, sq = ctx.align_batch(items, 8)
        ok_cost = []
        for k, (A, B, _) in enumerate(items):
            dt, dr = pose_error(Tq[k], cal[k // 4][2])
            if dt <= 0.05 and dr <= 0.5 and sq[k]["status"] in (cv.OK, cv.NOT_CONVERGED):
                ok_cost.append(cq[k])
        meta["c_thr"] = float(np.percentile(ok_cost, 95)) if ok_cost else math.inf
        meta["calibration_seeds"] = c_seeds
        _log("calibration: %d of %d aligned by plain 8-start, c_thr %.4g" % (len(ok_cost), len(items), meta["c_thr"]))
        save(a.out, net, losses, meta, a)
    _log("done (%.0f s)" % (time.perf_counter() - t0))
    ctx.close()


def save(path, net, losses, meta, a):
    meta = dict(meta)
    meta.update({"render_scale": a.render_scale, "batch": a.batch, "lr": a.lr, "cell": a.cell,
                 "final_loss": float(np.mean(losses[-100:])) if losses else None})
    meta.setdefault("c_thr", math.inf)
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp.npz"
    np.savez(tmp, params=net.get_params(), losses=np.asarray(losses, np.float32),
             meta=np.frombuffer(json.dumps(meta).encode(), np.uint8))
    os.replace(tmp, path)
    _log("saved %s: %s" % (path, json.dumps({k: v for k, v in meta.items() if k != "seeds"})))


def load(path=DEFAULT_OUT):
    """(params float32, meta dict) of a stored proposal network."""
    with np.load(path, allow_pickle=False) as z:
        return z["params"].astype(np.float32), json.loads(bytes(z["meta"]).decode())


if __name__ == "__main__":
    main()
