"""Trains the pose-proposal network on submap pairs that the mapping
pipeline itself generates, then stores the weights with the fallback cost
threshold.

Scenes: outdoor MAV-like workloads (120 x 80 m, 3000 frames 640x480, 0.1 m
voxels, 30 submaps of 100 frames) for a list of seeds.  Pairs: submaps i and
j (j = i+1..i+4) whose block overlap is at least 0.2, in both directions,
with the ground truth T_A_B from the generator's poses.  Training draws
re-framings of these pairs inside the library (covox_train_proposal: +-3 m
in x/y, +-0.5 m in z, +-180 deg yaw, +-2 deg roll/pitch of the prior).

The fallback threshold is the 95th percentile of the costs that plain
8-start alignment reaches on the pairs it aligns successfully (within 5 cm /
0.5 deg) in a calibration split (the last two scenes, priors perturbed by
+-0.5 m / +-10 deg yaw / +-2 deg roll and pitch).

Usage: python -m paper_2410_21149_amd.train_proposal [--scenes 36] [--out FILE]
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


def build_scene(cv, torch, ctx, seed, scale=1.0):
    """Maps one MAV scene into 30 gravity-aligned submaps with current
    ESDFs; returns (submaps, T_world_submap list) or None if the generator
    finds no path for this seed."""
    import scenegen as sg
    try:
        w = sg.mav(seed=seed, scale=scale)
    except RuntimeError:
        return None
    per = w.submap_every
    subs, Tws = [], []
    for k in range(w.n_frames // per):
        fr = torch.from_numpy(w.frames(k * per, (k + 1) * per)).cuda()
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


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--scenes", type=int, default=36)
    ap.add_argument("--seed0", type=int, default=101)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--cell", type=float, default=1.0)
    ap.add_argument("--net-seed", type=int, default=1)
    ap.add_argument("--block-capacity", type=int, default=8192, help="blocks per submap (submaps that overflow are skipped)")
    ap.add_argument("--render-scale", type=float, default=1.0,
                    help="render the training scenes at this fraction of 640x480 (same field of view)")
    ap.add_argument("--out", default=DEFAULT_OUT)
    a = ap.parse_args(argv)
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import torch

    import paper_2410_21149_amd as cv
    t0 = time.perf_counter()
    ctx = cv.Context(voxel_size=0.1, trunc_vox=4, max_range=10.0, d_max=3.0, block_capacity=a.block_capacity)
    scenes, seeds = [], []
    sd = a.seed0
    while len(scenes) < a.scenes:
        got = build_scene(cv, torch, ctx, sd, a.render_scale)
        if got is not None:
            scenes.append(got)
            seeds.append(sd)
            _log("scene seed %d: %d submaps (%.0f s)" % (sd, len(got[0]), time.perf_counter() - t0))
        sd += 1
    n_cal = 2 if len(scenes) > 4 else 0
    train, cal = [], []
    for k, (subs, Tws) in enumerate(scenes):
        for i, j, ov in block_pairs(ctx, subs, Tws, 0.1, min_overlap=0.2):
            T = np.linalg.inv(Tws[i]) @ Tws[j]
            dst = cal if k >= len(scenes) - n_cal else train
            dst.append((subs[i], subs[j], T))
            dst.append((subs[j], subs[i], np.linalg.inv(T)))
    _log("pairs: %d training, %d calibration" % (len(train), len(cal)))
    net = cv.Net(ctx, seed=a.net_seed)
    losses = []
    # step decay of the learning rate: 1, 1/3, 1/10 over the three thirds
    sched = [(a.steps - 2 * (a.steps // 3), a.lr), (a.steps // 3, a.lr / 3), (a.steps // 3, a.lr / 10)]
    chunk = 250
    done = 0
    for n_steps, lr in sched:
        left = n_steps
        while left > 0:
            m = min(chunk, left)
            L = ctx.train_proposal(net, train, steps=m, batch=a.batch, lr=lr, cell=a.cell, seed=1000 + done)
            losses.extend(L.tolist())
            done += m
            left -= m
            _log("step %d lr %.2g loss %.4f (%.0f s)" % (done, lr, float(np.mean(L[-50:])), time.perf_counter() - t0))
    # fallback threshold from plain 8-start on the calibration split
    c_thr = math.inf
    if cal:
        rng = np.random.default_rng(7)
        items = [(A, B, perturbed(rng, T)) for A, B, T in cal for _ in range(4)]
        Tq, cq, sq = ctx.align_batch(items, 8)
        ok_cost = []
        for k, (A, B, _) in enumerate(items):
            T_gt = cal[k // 4][2]
            dt, dr = pose_error(Tq[k], T_gt)
            if dt <= 0.05 and dr <= 0.5 and sq[k]["status"] in (cv.OK, cv.NOT_CONVERGED):
                ok_cost.append(cq[k])
        if ok_cost:
            c_thr = float(np.percentile(ok_cost, 95))
        _log("calibration: %d of %d aligned by plain 8-start, c_thr %.4g" % (len(ok_cost), len(items), c_thr))
    meta = {"seeds": seeds, "calibration_seeds": seeds[len(seeds) - n_cal:], "pairs_train": len(train),
            "render_scale": a.render_scale,
            "steps": a.steps, "batch": a.batch, "lr": a.lr, "cell": a.cell, "c_thr": c_thr,
            "final_loss": float(np.mean(losses[-100:])), "seconds": time.perf_counter() - t0}
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    np.savez(a.out, params=net.get_params(), losses=np.asarray(losses, np.float32),
             meta=np.frombuffer(json.dumps(meta).encode(), np.uint8))
    _log("saved %s: %s" % (a.out, json.dumps(meta)))
    ctx.close()


def load(path=DEFAULT_OUT):
    """(params float32, meta dict) of a stored proposal network."""
    with np.load(path, allow_pickle=False) as z:
        return z["params"].astype(np.float32), json.loads(bytes(z["meta"]).decode())


if __name__ == "__main__":
    main()
