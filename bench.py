#!/usr/bin/env python3
"""Benchmark of the covox hot path on one MI355X.

Step = the room workload mapped from scratch: 300 depth frames of 640x480
(fx = fy = 525), 5 cm voxels, truncation 4 voxels, ESDF (2 m) recomputed
after every frame -- projective integration (probe / scan / integrate
kernels) followed by the exact ESDF (page / x / y / z kernels) per frame.
The EDT passes of each frame's ESDF run on a second stream while the next
frame is integrated (covox_map_sequence).  The step is timed two ways: issued
call by call (W untimed, then K timed steps), and captured once as a HIP
graph (covox_graph_*) and replayed (W untimed, then K timed replays; skipped
with --no-graph).  value = frames per second of the faster of the two
(config.step_mode names it; inputs already resident in device memory);
config.eager_frames_per_s and config.graph_replay_frames_per_s give both.

Also reported on the same JSON line (every figure, with more, is also in the
full record printed to stderr and, with --detail-out PATH, written to PATH):
  roofline      the dominant kernel: the algorithmic bytes of the unit its
                launch belongs to (B_esdf per ESDF update, B_int per frame)
                divided by its mean duration from HIP events recorded around
                each of its launches, against 8 TB/s and against a 1 GiB
                device-to-device copy timed in the same run; and sum of
                bytes over sum of kernel time for the room step's ESDF and
                integration, the outdoor batched ESDF of 30 submaps and the
                outdoor mapping of 3000 frames;
  config.latency_per_frame  one frame integrated plus its ESDF, then a
                host synchronisation (median, p99, max over the sequence);
  cpu_baseline  the oracle (plain C, OpenMP over independent items) on the
                room workload on every host core, then on one thread over
                the same frames, with the CPU model and thread counts;
  aligns        ESDF alignment: room submap pairs, and outdoor pairs (every
                pair of the 30 submaps at block overlap 0.3 .. 0.9, both
                directions) -- pairs/s, success within 1 cm / 0.1 deg and
                5 cm / 0.5 deg, aligns/s within 1 cm / 0.1 deg;
  learned       learned proposal + refinement against plain 8-start on
                held-out outdoor pairs, with raw success counts;
  precision     FP32 and FP16 storage against the binary64 oracle on the
                room workload: D and phi errors, validity, site and band
                flips, the EDT alone on the same TSDF, and alignment poses.

--cfg4-align runs only the batched alignment of pairs drawn from several
outdoor scenes (and the accuracy-floor experiments) and prints that record.

Usage: python bench.py [--gpus 1] [--steps 3] [--warmup 1]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "TSDF+ESDF frames/s @640x480,5cm; submap-pair aligns/s at ≤1cm/0.1° err"
HBM_PEAK_GBS = 8000.0
OUTDOOR_TOL_RHO, OUTDOOR_TOL_THETA = 1e-5, 1e-6  # alignment stopping on the outdoor workload (m, rad)


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


ESDF_KINDS = ("esdf_page", "edt_x", "edt_y", "edt_z")
INTEGRATION_KINDS = ("probe", "scan", "integrate")


def frame_bytes(census, s_dw):
    """Algorithmic bytes per frame of the two parts of the step, from the
    per-frame counts of the workload (s_dw = bytes of D plus W per voxel: 8
    in FP32, 4 in FP16):
      integration  B_int  = 4 H W (depth) + 2 s_dw N_upd (state read and
                   written) + (s_dw 512 + 24) N_new (new blocks initialised;
                   key, index and slot)
      ESDF update  B_esdf = (s_dw + 4) 512 n_blocks (D and W read, phi written)
    Returns two lists, one value per frame."""
    HW = census["H"] * census["W"]
    b_int = [4 * HW + 2 * s_dw * u + (s_dw * 512 + 24) * n for u, n in zip(census["n_upd"], census["n_new"])]
    b_esdf = [(s_dw + 4) * 512 * nb for nb in census["n_blocks"]]
    return b_int, b_esdf


def unit_bytes(kind, census, s_dw):
    """Bytes of the unit of work one launch of `kind` belongs to, averaged
    over the frames: B_esdf for the ESDF kernels (one launch per update),
    B_int for the integration kernels (one launch per frame)."""
    b_int, b_esdf = frame_bytes(census, s_dw)
    b = b_esdf if kind in ESDF_KINDS else b_int
    return sum(b) / len(b)


def part_fraction(bytes_total, kernel_ms, peak=HBM_PEAK_GBS):
    """Sum of algorithmic bytes over the sum of kernel time, against peak."""
    if not kernel_ms or kernel_ms <= 0:
        return {"bytes": bytes_total, "kernel_ms": kernel_ms, "GBs": None, "frac": None}
    gbs = bytes_total / (kernel_ms * 1e-3) / 1e9
    return {"bytes": bytes_total, "kernel_ms": kernel_ms, "GBs": gbs, "frac": gbs / peak}


def measured_traffic(kind, tuning, census):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (profiles/room_hbm_traffic.md: FETCH_SIZE and WRITE_SIZE scaled by
    a copy of known size), or None when the kernel's source has changed since
    the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "room_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    table = None
    for line in open(path):
        if line.startswith("traffic_json: "):
            table = json.loads(line[len("traffic_json: "):])
    if not table:
        return None
    cols = (tuning or {}).get("edt_col_seg", 0) > 0  # column passes: x fused into y
    symbols = {"probe": "k_probe<float, true>", "scan": "k_scan", "integrate": "k_integrate<float, true>",
               "esdf_page": "k_page_sites<float, 1, true>", "edt_x": "k_edt_x<1>",
               "edt_y": "k_edt_xy<1>" if cols else "k_edt_y_col<1>",
               "edt_z": "k_edt_z_col<1>" if cols else "k_edt_z_vox<1>"}
    ent = table.get(symbols.get(kind, ""))
    if ent is None:
        return None
    src = os.path.join(ROOT, "paper_2410_21149_amd", "csrc", ent["source"])
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != ent["sha256"]:
        return None
    return ent["bytes_per_dispatch"]


def run_census(ctx, s, dev, w, np):
    """Untimed pass that records per-frame counts for the byte accounting."""
    ctx.submap_reset(s)
    info0 = ctx.submap_info(s)
    out = {k: [] for k in ("n_blocks", "n_new", "n_upd", "n_touched", "n_box", "n_dense")}
    prev_nb, prev_upd = 0, info0["n_updates"]
    vs = w.voxel_size
    for f in range(w.n_frames):
        ctx.integrate_depth(s, dev[f], w.cam.K, w.poses[f])
        ctx.update_esdf(s)
        info = ctx.submap_info(s)
        out["n_blocks"].append(info["n_blocks"])
        out["n_new"].append(info["n_blocks"] - prev_nb)
        out["n_upd"].append(info["n_updates"] - prev_upd)
        dims = [b - a + 1 for a, b in zip(info["bbox_min"], info["bbox_max"])]
        out["n_dense"].append(int(np.prod(dims)))
        out["n_box"].append(frustum_box_blocks(w, f, vs, np))
        out["n_touched"].append(0)
        prev_nb, prev_upd = info["n_blocks"], info["n_updates"]
    out["H"], out["W"] = w.cam.H, w.cam.W
    return out


def frustum_box_blocks(w, f, vs, np):
    """Blocks of the frustum box the probe kernel scans (same construction as
    the library: camera centre and far-plane corners at max_range + tau)."""
    T = w.poses[f]
    zf = w.cam.max_range + 4 * vs
    pts = [T[:3, 3]]
    for u in (-0.5, w.cam.W - 0.5):
        for v in (-0.5, w.cam.H - 0.5):
            pc = np.array([(u - w.cam.cx) / w.cam.fx * zf, (v - w.cam.cy) / w.cam.fy * zf, zf])
            pts.append(T[:3, :3] @ pc + T[:3, 3])
    P = np.array(pts)
    lo = np.floor(np.floor(P.min(0) / vs - 0.5) - 1) // 8
    hi = np.floor(np.ceil(P.max(0) / vs - 0.5) + 1) // 8
    return int(np.prod(hi - lo + 1))


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, frames, budget_s):
    """The oracle on a prefix of the room workload: integrate + ESDF after
    every frame, first with its parallel loops on every host core, then on
    one thread over the same frames (the results are the same bit for bit
    at any thread count).  About budget_s of CPU time in total."""
    import oracle as orc

    def run(threads, n_max, t_max):
        used = orc.set_threads(threads)
        ref = orc.Submap(orc.Params(vs=w.voxel_size, trunc_vox=4, max_range=w.cam.max_range, d_max=w.d_max))
        t0 = time.perf_counter()
        n = 0
        while n < n_max:
            ref.integrate(frames[n], w.cam.K, w.poses[n])
            ref.update_esdf()
            n += 1
            if time.perf_counter() - t0 > t_max:
                break
        return n, time.perf_counter() - t0, used

    n_all, t_all, cores = run(0, min(w.n_frames, len(frames)), 0.4 * budget_s)
    n_one, t_one, _ = run(1, n_all, 0.6 * budget_s)
    orc.set_threads(0)
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    return {"value": n_all / t_all, "unit": "frames/s", "cores": cores, "kind": "oracle",
            "sample": "first %d of %d room frames, integrate + ESDF after every frame, %.1f s on %d threads"
                      % (n_all, w.n_frames, t_all, cores),
            "single_thread": {"value": n_one / t_one, "frames": n_one, "seconds": t_one},
            "host": {"cpu_model": _cpu_model(), "nproc": os.cpu_count(), "affinity": affinity,
                     "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}}


def _pose_diff(Ta, Tb, np):
    """Translation difference (m) and rotation angle (rad) between two poses."""
    dt = float(np.linalg.norm(Ta[:3, 3] - Tb[:3, 3]))
    c = (np.trace(Ta[:3, :3] @ Tb[:3, :3].T) - 1) / 2
    return dt, math.acos(max(-1.0, min(1.0, c)))


def _field_errors(g, e64, np, vs, tau):
    """Errors of one GPU submap (export) against the binary64 oracle's, over
    the blocks both hold: |D - D64| and |phi - phi64| (max, RMS), validity
    decisions that differ (voxel-frame updates, as weight differences under
    unit weights), site flips (|D| <= vs with W > 0 on one side only) and
    band flips."""
    tab = {int(k): i for i, k in enumerate(e64["keys"])}
    rows = np.array([tab.get(int(k), -1) for k in g["keys"]])
    both = rows >= 0
    D, W = g["D"][both].astype(np.float64).ravel(), g["W"][both].astype(np.float64).ravel()
    P = g["phi"][both].astype(np.float64).ravel()
    D64, W64, P64 = (e64[k].reshape(-1, 512)[rows[both]].ravel() for k in ("D", "W", "phi"))
    obs, obs64 = W > 0, W64 > 0
    same = obs & obs64 & (W == W64)
    dD = np.abs(D - D64)[same]
    m = ~np.isnan(P) & ~np.isnan(P64)
    dP = np.abs(P - P64)[m]
    site, site64 = obs & (np.abs(D) <= vs), obs64 & (np.abs(D64) <= vs)
    band, band64 = obs & (np.abs(D) < tau), obs64 & (np.abs(D64) < tau)
    inb = m & band & band64
    return {"blocks": int(len(g["keys"])), "blocks_fp64": int(len(e64["keys"])),
            "blocks_one_side": int(np.count_nonzero(~both) + len(e64["keys"]) - int(both.sum())),
            "validity_flips": int(np.abs(W - W64).sum()), "observed_flips": int(np.count_nonzero(obs != obs64)),
            "voxels_compared": int(same.sum()),
            "D_max": float(dD.max(initial=0)), "D_rms": float(np.sqrt((dD ** 2).mean())) if dD.size else 0.0,
            "phi_max": float(dP.max(initial=0)), "phi_rms": float(np.sqrt((dP ** 2).mean())) if dP.size else 0.0,
            "phi_max_in_band": float(np.abs(P - P64)[inb].max(initial=0)),
            "phi_voxels_over_1e-4": int(np.count_nonzero(dP > 1e-4)),
            "site_flips": int(np.count_nonzero(site != site64)), "band_flips": int(np.count_nonzero(band != band64))}


def precision_bench(cv, torch, np, w, frames, dev, per=50):
    """Error statement of the binary32 and binary16 storage paths against the
    binary64 oracle on the room workload: the headline map (every frame into
    one submap, ESDF at the end) field by field, the same ESDF recomputed by
    the binary64 oracle from the GPU's own TSDF (which separates the EDT's
    arithmetic from the TSDF's rounding), and single-start alignment of the
    consecutive room submaps of `per` frames against the binary64 oracle's
    pose from the same start."""
    import oracle as orc
    import scenegen as sg
    F = w.n_frames
    P = dict(vs=w.voxel_size, trunc_vox=4, max_range=w.cam.max_range, d_max=w.d_max)
    vs, tau = w.voxel_size, 4 * w.voxel_size * (1 - 2.0 ** -10)
    orc.set_threads(0)
    t0 = time.perf_counter()
    r64 = orc.Submap(orc.Params(fp64=True, **P))
    nsub = F // per
    s64 = [orc.Submap(orc.Params(fp64=True, **P), w.poses[k * per]) for k in range(nsub)]
    for f in range(F):
        r64.integrate(frames[f], w.cam.K, w.poses[f])
        if f // per < nsub:
            s64[f // per].integrate(frames[f], w.cam.K, w.poses[f])
    r64.update_esdf()
    for sm in s64:
        sm.update_esdf()
    e64 = r64.export()
    rng = np.random.default_rng(77)
    pairs = []
    for i in range(nsub - 1):
        T_gt = np.linalg.inv(w.poses[i * per]) @ w.poses[(i + 1) * per]
        dT = np.eye(4)
        dT[:3, :3] = sg.rot_z(math.radians(rng.uniform(-5, 5)))
        dT[:3, 3] = rng.uniform(-0.1, 0.1, size=3)
        pairs.append((i, i + 1, T_gt @ dT))
    pose64 = [orc.align(s64[i], s64[j].iso_points(), T0)["T"] for i, j, T0 in pairs]
    out = {"workload": "room, %d frames: one submap (ESDF at the end); %d pairs of consecutive %d-frame submaps, "
                       "single-start Gauss-Newton from a perturbed start" % (F, len(pairs), per)}
    for name, prec in (("fp32", cv.FP32), ("fp16", cv.FP16)):
        ctx = cv.Context(voxel_size=w.voxel_size, trunc_vox=4, max_range=w.cam.max_range, d_max=w.d_max,
                         block_capacity=16384, precision=prec)
        s = ctx.submap_create()
        ctx.map_sequence(s, dev, w.cam.K, w.poses, esdf_every=0)
        ctx.update_esdf(s)
        g = ctx.export_blocks(s)
        r = _field_errors(g, e64, np, vs, tau)
        # the binary64 oracle's ESDF of the GPU's own TSDF: what is left is
        # the EDT's arithmetic alone
        imp = orc.Submap(orc.Params(fp64=True, **P))
        imp.import_blocks(g["keys"], g["D"].astype(np.float64), g["W"].astype(np.float64))
        imp.update_esdf()
        ei = imp.export()
        tab = {int(k): i for i, k in enumerate(ei["keys"])}
        rows = np.array([tab[int(k)] for k in g["keys"]])
        Pg, Pi = g["phi"].astype(np.float64).ravel(), ei["phi"].reshape(-1, 512)[rows].ravel()
        mm = ~np.isnan(Pg) & ~np.isnan(Pi)
        r["phi_max_same_tsdf"] = float(np.abs(Pg - Pi)[mm].max(initial=0))
        subs = [ctx.submap_create(w.poses[k * per]) for k in range(nsub)]
        for k in range(nsub):
            ctx.map_sequence(subs[k], dev[k * per:(k + 1) * per], w.cam.K, w.poses[k * per:(k + 1) * per],
                             esdf_every=0)
        T, _, _ = ctx.align_batch([(subs[i], subs[j], T0) for i, j, T0 in pairs], 1)
        d = [_pose_diff(Tg, T64, np) for Tg, T64 in zip(T, pose64)]
        r["pose_vs_fp64_max_t_m"] = max(x[0] for x in d)
        r["pose_vs_fp64_max_rot_rad"] = max(x[1] for x in d)
        out[name] = r
        ctx.close()
    out["cpu_s"] = time.perf_counter() - t0
    return out


def outdoor_pose_precision(cv, torch, np, w, ctx, subs, Tws, pairs, cand, n=3):
    """Pose difference of single-start alignment from the binary64 oracle's on
    outdoor pairs: the first n pairs of the benchmark set whose submaps are
    all distinct, each aligned from the same perturbed start by the GPU
    (FP32 and FP16 storage) and by the binary64 oracle (its own binary64 map
    of the same frames)."""
    import oracle as orc
    import scenegen as sg
    t0 = time.perf_counter()
    per = w.submap_every
    chosen, used = [], set()
    for k, (i, j, _) in enumerate(cand):
        if i in used or j in used:
            continue
        chosen.append((i, j, pairs[k][2]))
        used |= {i, j}
        if len(chosen) == n:
            break
    orc.set_threads(0)
    P = dict(vs=w.voxel_size, trunc_vox=4, max_range=w.cam.max_range, d_max=w.d_max, tol_rho=OUTDOOR_TOL_RHO,
             tol_theta=OUTDOOR_TOL_THETA)
    frames = {k: w.frames(k * per, (k + 1) * per) for k in used}
    ref = {}
    for k in used:
        r = orc.Submap(orc.Params(fp64=True, **P), Tws[k])
        for f in range(per):
            r.integrate(frames[k][f], w.cam.K, w.poses[k * per + f])
        r.update_esdf()
        ref[k] = r
    T64 = [orc.align(ref[i], ref[j].iso_points(), T0)["T"] for i, j, T0 in chosen]
    out = {"pairs": [[int(i), int(j)] for i, j, _ in chosen]}
    T32, _, _ = ctx.align_batch([(subs[i], subs[j], T0) for i, j, T0 in chosen], 1)
    c16 = cv.Context(voxel_size=w.voxel_size, trunc_vox=4, max_range=w.cam.max_range, d_max=w.d_max,
                     block_capacity=65536, precision=cv.FP16, tol_rho=OUTDOOR_TOL_RHO, tol_theta=OUTDOOR_TOL_THETA)
    s16 = {}
    for k in used:
        s16[k] = c16.submap_create(Tws[k])
        c16.map_sequence(s16[k], torch.from_numpy(frames[k]).cuda(), w.cam.K, w.poses[k * per:(k + 1) * per],
                         esdf_every=0)
    c16.update_esdf_batch(list(s16.values()))
    T16, _, _ = c16.align_batch([(s16[i], s16[j], T0) for i, j, T0 in chosen], 1)
    c16.close()
    for name, T in (("fp32", T32), ("fp16", T16)):
        d = [_pose_diff(a, b, np) for a, b in zip(T, T64)]
        out[name] = {"max_t_m": max(x[0] for x in d), "max_rot_rad": max(x[1] for x in d)}
    out["cpu_s"] = time.perf_counter() - t0
    return out


def align_bench(cv, torch, np, w, dev, reps=3):
    """Room submaps of 50 frames each (frame 0 of each submap defines its
    frame); overlapping pairs with seeded perturbations of the true relative
    pose (translation U[-0.5, 0.5]^3 m... scaled to the room: U[-0.1, 0.1] m,
    yaw U[-5, 5] deg, roll/pitch U[-1, 1] deg)."""
    import scenegen as sg
    ctx = cv.Context(voxel_size=w.voxel_size, trunc_vox=4, max_range=w.cam.max_range, d_max=w.d_max,
                     block_capacity=16384)
    per = 50
    subs, Tws = [], []
    for k in range(w.n_frames // per):
        T = w.poses[k * per]
        s = ctx.submap_create(T)
        ctx.map_sequence(s, dev[k * per:(k + 1) * per], w.cam.K, w.poses[k * per:(k + 1) * per], esdf_every=0)
        subs.append(s)
        Tws.append(T)
    pairs_idx = [(i, i + 1) for i in range(len(subs) - 1)] + [(i, i + 2) for i in range(len(subs) - 2)]
    rng = np.random.default_rng(44)
    pairs, gts = [], []
    for rep in range(16):
        for (i, j) in pairs_idx:
            T_gt = np.linalg.inv(Tws[i]) @ Tws[j]
            yaw = math.radians(rng.uniform(-5, 5))
            rp = np.radians(rng.uniform(-1, 1, size=2))
            dR = sg.rot_z(yaw) @ sg.rot_y(rp[0]) @ sg.rot_x(rp[1])
            dT = np.eye(4)
            dT[:3, :3] = dR
            dT[:3, 3] = rng.uniform(-0.1, 0.1, size=3)
            pairs.append((subs[i], subs[j], T_gt @ dT))
            gts.append(T_gt)
    ctx.align_batch(pairs[:2], 1)  # registration points extracted once per submap
    out = {"workload": "room submaps of 50 frames, %d pairs (%d distinct), perturbation 0.1 m / 5 deg yaw / 1 deg "
                       "roll-pitch" % (len(pairs), len(pairs_idx))}
    # Gauss-Newton (the default), then Levenberg-Marquardt on the same pairs
    for solver, prefix in ((cv.GAUSS_NEWTON, ""), (cv.LEVENBERG_MARQUARDT, "lm_")):
        ctx.set_params(align_solver=solver)
        for n_starts in (1, 8):
            tuning = ctx.autotune_align(pairs, n_starts)  # launch shape for this batch
            best = None
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                T, cost, st = ctx.align_batch(pairs, n_starts)
                dt = time.perf_counter() - t0
                best = dt if best is None else min(best, dt)
            ok = 0
            for Tg, Tt in zip(T, gts):
                et = np.linalg.norm(Tg[:3, 3] - Tt[:3, 3])
                c = (np.trace(Tg[:3, :3] @ Tt[:3, :3].T) - 1) / 2
                er = math.degrees(math.acos(max(-1.0, min(1.0, c))))
                ok += et <= 0.01 and er <= 0.1
            out["%sstarts_%d" % (prefix, n_starts)] = {"pairs_per_s": len(pairs) / best, "success": ok / len(pairs),
                                                        "ms": best * 1e3, **_solve_counts(st, np)}
    ctx.set_params(align_solver=cv.GAUSS_NEWTON)
    ctx.close()
    return out


def unpack_keys(k, np):
    """Block coordinates of packed keys ((bx+2^20)<<42 | (by+2^20)<<21 | bz+2^20)."""
    k = np.asarray(k, np.uint64)
    m = np.uint64(0x1FFFFF)
    return np.stack([((k >> np.uint64(42)) & m).astype(np.int64), ((k >> np.uint64(21)) & m).astype(np.int64),
                     (k & m).astype(np.int64)], axis=-1) - (1 << 20)


def block_overlap(keys_a, T_ws_a, keys_b, T_ws_b, vs, np):
    """|A blocks intersect T_gt B block centres| / min(|A|, |B|)."""
    ba = unpack_keys(keys_a, np)
    bb = unpack_keys(keys_b, np)
    T = np.linalg.inv(T_ws_a) @ T_ws_b
    cb = (bb + 0.5) * 8 * vs
    ca = cb @ T[:3, :3].T + T[:3, 3]
    ia = np.floor(ca / (8 * vs)).astype(np.int64)
    sa = set(map(tuple, ba))
    hit = sum(1 for t in map(tuple, ia) if t in sa)
    return hit / max(1, min(len(ba), len(bb)))


def mav_bench(cv, torch, np, reps=3, n_pairs=256, roofline_only=False):
    """MAV-scale outdoor workload: 3000 frames 640x480 cut into 30 submaps of
    100 frames (0.1 m voxels, ESDF to 3 m).  Reports the batched ESDF of all
    submaps (one launch per pass) and the batched alignment of overlapping
    submap pairs under perturbations of +-0.5 m, +-10 deg yaw, +-2 deg
    roll/pitch."""
    import scenegen as sg
    t0 = time.perf_counter()
    w = sg.mav()
    per = w.submap_every
    nsub = w.n_frames // per
    # Gauss-Newton stops at steps of 10 um / 1 urad here: with sigma = 0.002 z^2
    # the steps jitter well above the default 1e-7 m / 1e-8 rad at the noise
    # floor (a few cm), so the default would always run all 30 iterations.
    ctx = cv.Context(voxel_size=w.voxel_size, trunc_vox=4, max_range=w.cam.max_range, d_max=w.d_max,
                     block_capacity=65536, tol_rho=OUTDOOR_TOL_RHO, tol_theta=OUTDOOR_TOL_THETA)
    # all 3000 frames resident in HBM (3.7 GB), rendered on the host first
    frames = torch.empty((w.n_frames, w.cam.H, w.cam.W), dtype=torch.float32, device="cuda")
    for k in range(nsub):
        frames[k * per:(k + 1) * per].copy_(torch.from_numpy(w.frames(k * per, (k + 1) * per)))
    torch.cuda.synchronize()
    t_render = time.perf_counter() - t0
    Tws = [sg.gravity_aligned(w.poses[k * per]) for k in range(nsub)]
    subs = [ctx.submap_create(T) for T in Tws]

    def map_all():
        # each submap from scratch: frame batches of up to 64 frames, no ESDF
        for k in range(nsub):
            ctx.submap_reset(subs[k])
            ctx.map_sequence(subs[k], frames[k * per:(k + 1) * per], w.cam.K, w.poses[k * per:(k + 1) * per],
                             esdf_every=0)

    map_all()
    torch.cuda.synchronize()
    ctx.timing_enable(["probe", "scan", "integrate"])
    map_all()
    torch.cuda.synchronize()
    map_kernels = {k: v[0] for k, v in ctx.timing_get().items() if v[1]}
    ctx.timing_enable([])
    best_map = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        map_all()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        best_map = dt if best_map is None else min(best_map, dt)
    n_upd = sum(ctx.submap_info(s)["n_updates"] for s in subs)
    n_blk = sum(ctx.submap_info(s)["n_blocks"] for s in subs)
    # B_int summed over the frames: depth once per frame, two state accesses
    # per voxel update, new blocks initialised once (FP32 state: 8 B per voxel)
    b_map = 4 * w.cam.H * w.cam.W * w.n_frames + 2 * 8 * n_upd + (8 * 512 + 24) * n_blk
    mapping = {"frames": w.n_frames, "frames_per_s": w.n_frames / best_map, "ms": best_map * 1e3,
               "voxel_updates": int(n_upd), "voxel_updates_per_s": n_upd / best_map, "kernel_ms": map_kernels,
               "roofline": part_fraction(b_map, sum(map_kernels.values())),
               "wall_GBs": b_map / best_map / 1e9}
    mapping["concurrent"] = concurrent_mapping(cv, torch, np, w, frames, Tws, ctx, subs, b_map, reps)
    large = sweep = None
    if not roofline_only:
        large = large_submap_esdf_bench(cv, torch, np, w, frames[:600], reps)
        sweep = voxel_sweep_bench(cv, torch, np, w, frames[:per], Tws[0])
    del frames
    t_build = time.perf_counter() - t0
    nblk = [ctx.submap_info(s)["n_blocks"] for s in subs]
    # batched ESDF of every submap, pass shapes chosen by the autotuner; every
    # timed update recomputes every block (as when all submaps are finalised)
    tuning = ctx.autotune_esdf(subs)
    ctx.set_tuning(esdf_full_recompute=1)
    ctx.timing_enable(["esdf_page", "edt_x", "edt_y", "edt_z"])
    ctx.update_esdf_batch(subs)
    torch.cuda.synchronize()
    ctx.timing_get()
    ctx.timing_enable(["esdf_page", "edt_x", "edt_y", "edt_z"])
    t1 = time.perf_counter()
    for _ in range(reps):
        ctx.update_esdf_batch(subs)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t1) / reps
    tk = ctx.timing_get()
    ctx.timing_enable([])
    kern = {k: v[0] / reps for k, v in tk.items() if v[1]}
    kms = sum(kern.values())
    b_esdf = 12 * 512 * sum(nblk)  # B_esdf: D and W read, phi written, every voxel of every submap
    esdf = {"submaps": nsub, "blocks_total": int(sum(nblk)), "blocks_min": int(min(nblk)), "blocks_max": int(max(nblk)),
            "ms_per_batch": wall * 1e3, "kernel_ms": kern, "roofline": part_fraction(b_esdf, kms),
            "voxels_per_s": 512 * sum(nblk) / (kms * 1e-3), "tuning": tuning}
    if roofline_only:
        ctx.close()
        return {"workload": "outdoor 120x80 m, 3000 frames 640x480 fx=fy=380, 0.1 m voxels, 30 submaps of 100 "
                            "frames (mapping and batched ESDF only)",
                "build_s": t_build, "render_s": t_render, "mapping": mapping, "esdf_batch": esdf}
    # overlapping pairs
    keys = [ctx.export_blocks(s)["keys"] for s in subs]
    # every submap pair of the trajectory (loop closures included) whose block
    # overlap is within 0.3 .. 0.9, in both directions (points from one,
    # field from the other)
    cand = []
    for i in range(nsub):
        for j in range(i + 1, nsub):
            ov = block_overlap(keys[i], Tws[i], keys[j], Tws[j], w.voxel_size, np)
            if 0.3 <= ov <= 0.9:
                cand.append((i, j, ov))
                cand.append((j, i, ov))
    def make_pairs(seed, tilt_deg):
        rng = np.random.default_rng(seed)
        pairs, gts = [], []
        for k in range(n_pairs):
            i, j, _ = cand[k % len(cand)]
            T_gt = np.linalg.inv(Tws[i]) @ Tws[j]
            dR = sg.rot_z(math.radians(rng.uniform(-10, 10))) @ sg.rot_y(math.radians(rng.uniform(-tilt_deg, tilt_deg))) \
                @ sg.rot_x(math.radians(rng.uniform(-tilt_deg, tilt_deg)))
            dT = np.eye(4)
            dT[:3, :3] = dR
            dT[:3, 3] = rng.uniform(-0.5, 0.5, size=3)
            pairs.append((subs[i], subs[j], T_gt @ dT))
            gts.append(T_gt)
        return pairs, gts

    def run_pairs(pairs, gts, n_starts):
        tuning = ctx.autotune_align(pairs, n_starts)
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            T, cost, st = ctx.align_batch(pairs, n_starts)
            dt = time.perf_counter() - t2
            best = dt if best is None else min(best, dt)
        ok, ok5, errs = 0, 0, []
        for Tg, Tt in zip(T, gts):
            et = np.linalg.norm(Tg[:3, 3] - Tt[:3, 3])
            c = (np.trace(Tg[:3, :3] @ Tt[:3, :3].T) - 1) / 2
            er = math.degrees(math.acos(max(-1.0, min(1.0, c))))
            ok += et <= 0.01 and er <= 0.1
            ok5 += et <= 0.05 and er <= 0.5
            errs.append(et)
        return {"pairs_per_s": n_pairs / best, "success": ok / n_pairs, "success_5cm": ok5 / n_pairs,
                "aligned_per_s": ok / best, "median_t_err_m": float(np.median(errs)),
                "ms": best * 1e3, **_solve_counts(st, np), "tuning": tuning}

    pairs, gts = make_pairs(4, 2.0)
    ctx.align_batch(pairs[:1], 1)
    align = {"pairs": n_pairs, "distinct_pairs": len(cand),
             "tol_rho_m": OUTDOOR_TOL_RHO, "tol_theta_rad": OUTDOOR_TOL_THETA,
             "overlap_range": [float(min(c[2] for c in cand)), float(max(c[2] for c in cand))]}
    for n_starts in (1, 8):
        align["starts_%d" % n_starts] = run_pairs(pairs, gts, n_starts)
    align["precision"] = outdoor_pose_precision(cv, torch, np, w, ctx, subs, Tws, pairs[:len(cand)], cand)
    ctx.set_params(align_solver=cv.LEVENBERG_MARQUARDT)  # the same pairs under Levenberg-Marquardt
    for n_starts in (1, 8):
        align["lm_starts_%d" % n_starts] = run_pairs(pairs, gts, n_starts)
    ctx.set_params(align_solver=cv.GAUSS_NEWTON)
    # gravity-aligned priors (roll and pitch known, as from an IMU): the
    # 4-DoF estimate (translation and yaw) beside the 6-DoF one on the same pairs
    pairs_g, gts_g = make_pairs(5, 0.0)
    align_4dof = {"prior": "+-0.5 m, +-10 deg yaw, roll/pitch exact"}
    for dof in (6, 4):
        ctx.set_params(align_dof=dof)
        for n_starts in (1, 8):
            align_4dof["dof%d_starts_%d" % (dof, n_starts)] = run_pairs(pairs_g, gts_g, n_starts)
    ctx.set_params(align_dof=6)
    align["gravity_aligned_priors"] = align_4dof
    # pose graph: every pair within three submaps that shares at least 10 % of its blocks
    cand_pgo = []
    for i in range(nsub):
        for j in range(i + 1, min(nsub, i + 4)):
            ov = block_overlap(keys[i], Tws[i], keys[j], Tws[j], w.voxel_size, np)
            if ov >= 0.1:
                cand_pgo.append((i, j, ov))
    pose_graph = pgo_bench(cv, torch, np, ctx, subs, Tws, cand_pgo, reps)
    ctx.close()
    learned = learned_bench(cv, torch, np)
    return {"workload": "outdoor 120x80 m, 3000 frames 640x480 fx=fy=380, 0.1 m voxels, 30 submaps of 100 frames",
            "build_s": t_build, "render_s": t_render, "mapping": mapping, "esdf_batch": esdf,
            "esdf_large_submap": large, "voxel_sweep": sweep, "align": align, "pose_graph": pose_graph,
            "learned": learned}


def concurrent_mapping(cv, torch, np, w, frames, Tws, ctx0, subs0, b_map, reps, n_ctx=4):
    """The same 3000 frames mapped from n_ctx contexts at once, each on a
    stream of its own and driven by a host thread of its own (submap k on
    context k mod n_ctx), as independent submaps may be built.  Wall time of
    the whole mapping; the roofline fraction is the algorithmic bytes over
    that wall time (the kernels of different streams overlap, so their sum
    is no measure here).  Every submap's blocks, D and W equal those of the
    single-context run."""
    import concurrent.futures
    per = w.submap_every
    nsub = len(Tws)
    ctxs = []
    for _ in range(n_ctx):
        c = cv.Context(voxel_size=w.voxel_size, trunc_vox=4, max_range=w.cam.max_range, d_max=w.d_max,
                       block_capacity=65536)
        c.set_stream(torch.cuda.Stream())
        ctxs.append(c)
    torch.cuda.synchronize()
    subs = [ctxs[k % n_ctx].submap_create(Tws[k]) for k in range(nsub)]
    pool = concurrent.futures.ThreadPoolExecutor(n_ctx)

    def run(ci):
        c = ctxs[ci]
        for k in range(ci, nsub, n_ctx):
            c.submap_reset(subs[k])
            c.map_sequence(subs[k], frames[k * per:(k + 1) * per], w.cam.K, w.poses[k * per:(k + 1) * per],
                           esdf_every=0)
        c.sync()

    def map_all():
        list(pool.map(run, range(n_ctx)))

    map_all()
    best = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        map_all()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        best = dt if best is None else min(best, dt)
    same = True
    for k in range(nsub):
        a, b = ctx0.export_blocks(subs0[k]), ctxs[k % n_ctx].export_blocks(subs[k])
        same = same and all(np.array_equal(a[q], b[q]) for q in ("keys", "D", "W"))
    assert same, "concurrent mapping differs from the single-context run"
    pool.shutdown()
    for c in ctxs:
        c.close()
    gbs = b_map / best / 1e9
    return {"contexts": n_ctx, "frames_per_s": w.n_frames / best, "ms": best * 1e3, "wall_GBs": gbs,
            "frac_wall": gbs / HBM_PEAK_GBS, "same_blocks_D_W": same}


def _solve_counts(stats, np):
    """Per-pair means of the pose updates applied (Levenberg-Marquardt: steps
    taken) and of the binary64 solves made (rejected steps included), and the
    fraction of pairs that ended converged."""
    return {"mean_iterations": float(np.mean([x["iterations"] for x in stats])),
            "mean_solves": float(np.mean([x["solves"] for x in stats])),
            "converged": float(np.mean([x["status"] == 0 for x in stats]))}


def _pose_errors(T, gts, np):
    """Translation (m) and rotation (deg) error of each pose against the truth."""
    et, er = [], []
    for Tg, Tt in zip(T, gts):
        et.append(float(np.linalg.norm(Tg[:3, 3] - Tt[:3, 3])))
        c = (np.trace(Tg[:3, :3] @ Tt[:3, :3].T) - 1) / 2
        er.append(math.degrees(math.acos(max(-1.0, min(1.0, c)))))
    return np.array(et), np.array(er)


def cfg4_align_bench(cv, torch, np, seeds=(40, 41, 42, 43, 44), n_pairs=256, reps=3, experiment_seeds=2):
    """Batched alignment on submap pairs of several outdoor scenes: each seed's
    3000-frame trajectory is cut into 30 submaps of 100 frames (0.1 m voxels,
    ESDF to 3 m); every pair of submaps of a scene whose block overlap lies in
    0.3 .. 0.9 enters in both directions; n_pairs distinct pairs are drawn
    (all of them when there are fewer) and perturbed by U[-0.5, 0.5]^3 m,
    U[-10, 10] deg yaw and U[-2, 2] deg roll and pitch.  Reports pairs/s and
    the success fraction at 1 cm / 0.1 deg and at 5 cm / 0.5 deg, for 1 and 8
    starts.  Two experiments on the pairs of the first experiment_seeds
    scenes name what sets the accuracy floor: the same pairs mapped from
    noise-free frames, and mapped from the same noisy frames by raycasting."""
    import scenegen as sg
    t0 = time.perf_counter()
    per = 100

    def build(ctx, w, Tws, cache=None):
        subs = []
        for k in range(len(Tws)):
            fr = cache[k] if cache is not None else torch.from_numpy(w.frames(k * per, (k + 1) * per)).cuda()
            s = ctx.submap_create(Tws[k])
            ctx.map_sequence(s, fr, w.cam.K, w.poses[k * per:(k + 1) * per], esdf_every=0)
            subs.append(s)
        ctx.update_esdf_batch(subs)
        return subs

    def make_ctx(**kw):
        return cv.Context(voxel_size=0.1, trunc_vox=4, max_range=10.0, d_max=3.0, block_capacity=16384,
                          tol_rho=OUTDOOR_TOL_RHO, tol_theta=OUTDOOR_TOL_THETA, **kw)

    ctx = make_ctx()
    scenes = []
    sd = seeds[0] - 1
    while len(scenes) < len(seeds):
        sd += 1
        try:
            w = sg.mav(seed=sd)
        except RuntimeError:  # the generator found no collision-free path for this seed
            continue
        nsub = w.n_frames // per
        Tws = [sg.gravity_aligned(w.poses[k * per]) for k in range(nsub)]
        keep = len(scenes) < experiment_seeds
        frames = [torch.from_numpy(w.frames(k * per, (k + 1) * per)).cuda() for k in range(nsub)] if keep else None
        subs = build(ctx, w, Tws, frames)
        keys = [ctx.export_blocks(s)["keys"] for s in subs]
        cand = []
        for i in range(nsub):
            for j in range(i + 1, nsub):
                ov = block_overlap(keys[i], Tws[i], keys[j], Tws[j], w.voxel_size, np)
                if 0.3 <= ov <= 0.9:
                    cand += [(i, j, ov), (j, i, ov)]
        scenes.append({"seed": sd, "w": w, "Tws": Tws, "subs": subs, "cand": cand, "frames": frames})
    t_build = time.perf_counter() - t0
    rng = np.random.default_rng(4)
    allc = [(si, i, j, ov) for si, sc in enumerate(scenes) for (i, j, ov) in sc["cand"]]
    order = rng.permutation(len(allc))[:n_pairs]
    chosen = [allc[k] for k in order]
    items = []
    for (si, i, j, ov) in chosen:
        sc = scenes[si]
        T_gt = np.linalg.inv(sc["Tws"][i]) @ sc["Tws"][j]
        dT = np.eye(4)
        dT[:3, :3] = sg.rot_z(math.radians(rng.uniform(-10, 10))) @ sg.rot_y(math.radians(rng.uniform(-2, 2))) \
            @ sg.rot_x(math.radians(rng.uniform(-2, 2)))
        dT[:3, 3] = rng.uniform(-0.5, 0.5, size=3)
        items.append((si, i, j, T_gt, T_gt @ dT))

    def run(c, subs_of, sel, n_starts):
        pairs = [(subs_of(si)[i], subs_of(si)[j], T0) for (si, i, j, _, T0) in sel]
        gts = [T_gt for (_, _, _, T_gt, _) in sel]
        c.autotune_align(pairs, n_starts)
        best, res = None, None
        for _ in range(reps):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            res = c.align_batch(pairs, n_starts)
            dt = time.perf_counter() - t1
            best = dt if best is None else min(best, dt)
        et, er = _pose_errors(res[0], gts, np)
        n = len(sel)
        ok1 = int(np.count_nonzero((et <= 0.01) & (er <= 0.1)))
        ok5 = int(np.count_nonzero((et <= 0.05) & (er <= 0.5)))
        return {"pairs": n, "pairs_per_s": n / best, "ms": best * 1e3, "success": ok1 / n, "successes": ok1,
                "success_5cm": ok5 / n, "successes_5cm": ok5, "aligned_per_s": ok1 / best,
                "median_t_err_m": float(np.median(et)), "median_rot_err_deg": float(np.median(er)),
                **_solve_counts(res[2], np)}

    out = {"workload": "outdoor scenes seeds %s, 30 submaps of 100 frames each, pairs at block overlap 0.3-0.9 "
                       "in both directions, perturbation 0.5 m / 10 deg yaw / 2 deg roll-pitch"
                       % [sc["seed"] for sc in scenes],
           "distinct_pairs_available": len(allc), "pairs": len(items),
           "pairs_per_scene": [len(sc["cand"]) for sc in scenes],
           "overlap_range": [float(min(c[3] for c in chosen)), float(max(c[3] for c in chosen))],
           "build_s": t_build}
    for n_starts in (1, 8):
        out["starts_%d" % n_starts] = run(ctx, lambda si: scenes[si]["subs"], items, n_starts)
    # the accuracy floor: the pairs of the first scenes, mapped three ways
    sel = [it for it in items if it[0] < experiment_seeds]
    exp = {"pairs": len(sel), "seeds": [sc["seed"] for sc in scenes[:experiment_seeds]]}
    exp["noisy_projective"] = run(ctx, lambda si: scenes[si]["subs"], sel, 1)
    cr = make_ctx(integrator=cv.RAYCAST)
    rsubs = [build(cr, scenes[si]["w"], scenes[si]["Tws"], scenes[si]["frames"]) for si in range(experiment_seeds)]
    exp["noisy_raycast"] = run(cr, lambda si: rsubs[si], sel, 1)
    cr.close()
    cn = make_ctx()
    nsubs = []
    for si in range(experiment_seeds):
        wc = sg.mav(seed=scenes[si]["seed"], noise=False)
        nsubs.append(build(cn, wc, scenes[si]["Tws"]))
    exp["noise_free_projective"] = run(cn, lambda si: nsubs[si], sel, 1)
    cn.close()
    out["accuracy_floor"] = exp
    out["total_s"] = time.perf_counter() - t0
    ctx.close()
    return out


def _success(T, gts, np, bound_t, bound_deg):
    ok = 0
    for Tg, Tt in zip(T, gts):
        et = np.linalg.norm(Tg[:3, 3] - Tt[:3, 3])
        c = (np.trace(Tg[:3, :3] @ Tt[:3, :3].T) - 1) / 2
        ok += et <= bound_t and math.degrees(math.acos(max(-1.0, min(1.0, c)))) <= bound_deg
    return ok / max(1, len(gts))


def _linear_fit(x, y, np):
    """Least-squares line y = a + b x and its coefficient of determination."""
    x, y = np.asarray(x, float), np.asarray(y, float)
    b, a = np.polyfit(x, y, 1)
    res = y - (a + b * x)
    r2 = 1.0 - (res @ res) / max(((y - y.mean()) ** 2).sum(), 1e-300)
    return a, b, r2


def voxel_sweep_bench(cv, torch, np, w, frames, T_ws, sizes=(0.20, 0.15, 0.10, 0.075, 0.05), reps=2):
    """Integration time against the number of updated voxels (Sec. IV, TSDF
    timings: raycasting scales almost linearly with the voxel count): the
    first submap's frames of the outdoor sequence integrated at five voxel
    sizes, by raycasting (carved from the optical centre, as in the paper)
    and by projection mapping.  Per size: ms per frame (best of reps after a
    warm-up pass), voxel updates per frame, blocks; per integrator: the
    least-squares line ms = a + b * updates and its R^2."""
    out = {}
    F = frames.shape[0]
    poses = w.poses[:F]
    for name, kw in (("raycast_carve", dict(integrator=cv.RAYCAST, ray_carve=1)),
                     ("projective", dict(integrator=cv.PROJECTIVE))):
        rows = []
        for vs in sizes:
            cap = int(min(1 << 20, max(16384, 16384 * (0.10 / vs) ** 3)))
            row = {"voxel_size": vs, "block_capacity": cap}
            try:
                # no ESDF here; its range is capped at 40 voxels only to keep the
                # parameters valid at the finest size
                ctx = cv.Context(voxel_size=vs, trunc_vox=4, max_range=w.cam.max_range,
                                 d_max=min(w.d_max, 40 * vs), block_capacity=cap, **kw)
            except cv.CovoxError as e:
                row["error"] = str(e)
                rows.append(row)
                continue
            s = ctx.submap_create(T_ws)
            try:
                best = None
                for k in range(reps + 1):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    ctx.submap_reset(s)
                    ctx.map_sequence(s, frames, w.cam.K, poses, esdf_every=0)
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - t0
                    if k > 0:
                        best = dt if best is None else min(best, dt)
                info = ctx.submap_info(s)
                row.update({"ms_per_frame": best * 1e3 / F, "voxel_updates_per_frame": info["n_updates"] / F,
                            "blocks": info["n_blocks"],
                            "ns_per_voxel_update": best * 1e9 / max(info["n_updates"], 1)})
            except cv.CovoxError as e:
                row["error"] = str(e)
            ctx.close()
            rows.append(row)
        ok = [r for r in rows if "ms_per_frame" in r]
        fit = None
        if len(ok) >= 3:
            a, b, r2 = _linear_fit([r["voxel_updates_per_frame"] for r in ok], [r["ms_per_frame"] for r in ok], np)
            fit = {"intercept_ms": a, "ns_per_update": b * 1e6, "r2": r2}
        out[name] = {"sizes": rows, "linear_fit": fit}
    out["frames"] = F
    return out


def hash_bench(cv, torch, np, cap_log2=26, loads=(0.25, 0.40, 0.55, 0.70, 0.85), batch=1 << 20):
    """Hash-table stress test (Sec. IV): a table of 2^26 slots (the capacity
    is a power of two, so the load factor is set by the key count: 16.8 M to
    57 M keys) filled from empty to each load factor with distinct random
    keys (seed 7) in batches of 2^20 keys.  Per load factor: keys per second
    over the whole fill (kernel time, HIP events), ms of the last batch (the
    fullest table), the longest and the mean probe."""
    import scenegen as sg
    cap = 1 << cap_log2
    n_max = int(max(loads) * cap)
    keys = torch.from_numpy(sg.hash_keys(n_max, seed=7).view(np.int64)).cuda()
    tk = torch.empty(cap, dtype=torch.int64, device="cuda")
    tv = torch.empty(cap, dtype=torch.int32, device="cuda")
    ctx = cv.Context(block_capacity=64)
    out = {"capacity": cap, "batch_keys": batch, "loads": []}
    for lf in loads:
        n = int(lf * cap)
        nb = (n + batch - 1) // batch
        stats = torch.zeros(nb, 3, dtype=torch.int64, device="cuda")
        best = None
        for rep in range(3):
            tk.fill_(-1)
            stats.zero_()
            torch.cuda.synchronize()
            ctx.timing_enable(["hash"])
            for j in range(nb):
                if j == nb - 1:
                    last = ctx.timing_get()["hash"][0]
                    ctx.timing_enable(["hash"])
                b0 = j * batch
                ctx.hash_insert(tk, tv, b0, keys[b0:min(n, b0 + batch)], stats[j], val_base=b0)
            ms_last = ctx.timing_get()["hash"][0]
            ms = last + ms_last if nb > 1 else ms_last
            ctx.timing_enable([])
            if best is None or ms < best[0]:
                best = (ms, ms_last)
        st = stats.cpu().numpy()
        out["loads"].append({"load_factor": lf, "keys": n, "mkeys_per_s": n / (best[0] * 1e-3) / 1e6,
                             "ms_fill": best[0], "ms_last_batch": best[1],
                             "last_batch_keys": n - (nb - 1) * batch,
                             "max_probe": int(st[:, 0].max()), "mean_probe": float(st[:, 1].sum()) / n,
                             "failed": int(st[:, 2].sum())})
    ctx.close()
    del keys, tk, tv
    return out


def large_submap_esdf_bench(cv, torch, np, w, frames, reps=2, every=20):
    """One large outdoor submap (the first 600 frames, about 80 m of path)
    with an ESDF update after every 20 frames: the exact EDT recomputing the
    whole box each time, the exact EDT recomputing only the blocks near the
    blocks changed since the last update (the same bits), and the wavefront
    (Sec. III-E).  Reports the ESDF time per update (mapping with updates
    minus mapping without) and the wavefront's error against the exact field
    at the end."""
    import scenegen as sg
    F = len(frames)
    T_ws = sg.gravity_aligned(w.poses[0])
    out, fields = {"frames": F, "update_every": every}, {}
    # exact: per-block passes (every update recomputes the whole submap);
    # exact_dirty_region: column passes (segments of 16 blocks), each update
    # recomputing only the blocks near the blocks changed since the last one
    for name, mode, seg in (("exact", cv.ESDF_EXACT, 0), ("exact_dirty_region", cv.ESDF_EXACT, 16),
                            ("wavefront", cv.ESDF_WAVEFRONT, 0)):
        ctx = cv.Context(voxel_size=w.voxel_size, trunc_vox=4, max_range=w.cam.max_range, d_max=w.d_max,
                         block_capacity=131072, esdf_mode=mode)
        ctx.set_tuning(edt_col_seg=seg)
        s = ctx.submap_create(T_ws)
        times = {}
        for label, e in (("map_only", 0), ("map_esdf", every)):
            best = None
            for k in range(reps + 1):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.submap_reset(s)
                ctx.map_sequence(s, frames, w.cam.K, w.poses[:F], esdf_every=e)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                if k > 0:
                    best = dt if best is None else min(best, dt)
            times[label] = best
        n_upd = F // every
        info = ctx.submap_info(s)
        out[name] = {"ms_per_update": (times["map_esdf"] - times["map_only"]) * 1e3 / n_upd,
                     "map_esdf_ms": times["map_esdf"] * 1e3, "map_only_ms": times["map_only"] * 1e3,
                     "blocks": info["n_blocks"]}
        fields[name] = ctx.export_blocks(s)
        ctx.close()
    assert np.array_equal(fields["exact"]["phi"], fields["exact_dirty_region"]["phi"], equal_nan=True)
    a, b = fields["exact"], fields["wavefront"]
    m = ~np.isnan(a["phi"])
    d = np.abs(a["phi"][m].astype(np.float64) - b["phi"][m])
    out["wavefront_vs_exact"] = {"observed_voxels": int(m.sum()), "equal_fraction": float((d == 0).mean()),
                                 "max_abs_m": float(d.max(initial=0)), "rms_m": float(np.sqrt((d ** 2).mean()))}
    out["speedup_wavefront"] = out["exact"]["ms_per_update"] / max(out["wavefront"]["ms_per_update"], 1e-9)
    out["speedup_dirty_region"] = out["exact"]["ms_per_update"] / max(out["exact_dirty_region"]["ms_per_update"],
                                                                       1e-9)
    return out


def pgo_bench(cv, torch, np, ctx, subs, Tws, cand, reps=2):
    """Submap pose-graph optimisation (Eq. 1) over the 30 outdoor submaps:
    odometry between consecutive submaps with noise (0.1 m horizontal,
    0.05 m vertical, 0.3 deg yaw per step, the factor sigmas), poses started
    at dead reckoning from it, registration terms for every pair within
    three submaps sharing at least 10 % of its blocks, in both directions.  Reports the position / yaw RMS error against the
    ground truth before and after, LM iterations and the wall time."""
    n = len(subs)
    x_true = np.array([[T[0, 3], T[1, 3], T[2, 3], math.atan2(T[1, 0], T[0, 0])] for T in Tws])

    def rel(xi, xj):
        c, s = math.cos(xi[3]), math.sin(xi[3])
        d = xj[:3] - xi[:3]
        return np.array([c * d[0] + s * d[1], -s * d[0] + c * d[1], d[2], xj[3] - xi[3]])

    rng = np.random.default_rng(7)
    sig = np.array([0.1, 0.1, 0.05, math.radians(0.3)])
    facs, x0 = [], np.zeros_like(x_true)
    x0[0] = x_true[0]
    for k in range(n - 1):
        z = rel(x_true[k], x_true[k + 1]) + rng.normal(size=4) * sig
        facs.append(dict(i=k, j=k + 1, z=z, sigma=sig))
        c, s = math.cos(x0[k, 3]), math.sin(x0[k, 3])
        x0[k + 1, :3] = x0[k, :3] + np.array([c * z[0] - s * z[1], s * z[0] + c * z[1], z[2]])
        x0[k + 1, 3] = x0[k, 3] + z[3]
    pairs = [(i, j) for (i, j, _) in cand] + [(j, i) for (i, j, _) in cand]

    def err(x):
        dp = np.linalg.norm(x[:, :3] - x_true[:, :3], axis=1)
        dy = np.degrees(np.abs(np.angle(np.exp(1j * (x[:, 3] - x_true[:, 3])))))
        return float(np.sqrt(np.mean(dp ** 2))), float(np.sqrt(np.mean(dy ** 2)))

    ctx.pgo_solve(subs, x0, pairs, facs, max_iter=2)  # registration points extracted once
    best, out = None, None
    for _ in range(reps):
        ctx.timing_enable(["align", "pgo"])
        t0 = time.perf_counter()
        x, st = ctx.pgo_solve(subs, x0, pairs, facs, sigma_reg=0.05, max_iter=20)
        dt = time.perf_counter() - t0
        tk = ctx.timing_get()
        ctx.timing_enable([])
        if best is None or dt < best:
            best, out = dt, (x, st, tk)
    x, st, tk = out
    e0, e1 = err(x0), err(x)
    return {"submaps": n, "registration_terms": len(pairs), "odometry_terms": len(facs),
            "rms_position_error_m": {"dead_reckoning": e0[0], "optimised": e1[0]},
            "rms_yaw_error_deg": {"dead_reckoning": e0[1], "optimised": e1[1]},
            "lm_iterations": st["iterations"], "accepted": st["accepted"], "cg_iterations": st["cg_iterations"],
            "ms": best * 1e3, "ms_per_lm_iteration": best * 1e3 / max(st["iterations"], 1),
            "kernel_ms": {k: v[0] for k, v in tk.items() if v[1]}}


def learned_bench(cv, torch, np, n_items=1024, reps=3, min_distinct=256, seed0=4):
    """Learned proposal + refinement against plain 8-start on held-out pairs:
    outdoor scenes from seed seed0 on (no training or calibration seed
    among them), built until they give at least min_distinct directed pairs
    with block overlap >= 0.2 (j = i+1..i+4, both directions), each pair
    re-framed like the training data (+-3 m x/y, +-0.5 m z, +-180 deg yaw
    about the summary grid centre, +-2 deg roll/pitch); n_items items drawn
    round-robin over the pairs."""
    import importlib.util
    path = os.path.join(ROOT, "paper_2410_21149_amd", "data", "proposal_mav.npz")
    if not os.path.exists(path):
        return {"skipped": "no trained proposal weights at " + os.path.relpath(path, ROOT)}
    spec = importlib.util.spec_from_file_location("_train_proposal", os.path.join(ROOT, "paper_2410_21149_amd",
                                                                                    "train_proposal.py"))
    tp = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(tp)
    params, meta = tp.load(path)
    t0 = time.perf_counter()
    ctx = cv.Context(voxel_size=0.1, trunc_vox=4, max_range=10.0, d_max=3.0, block_capacity=16384,
                     tol_rho=OUTDOOR_TOL_RHO, tol_theta=OUTDOOR_TOL_THETA)
    net = cv.Net(ctx, seed=1)
    net.set_params(params)
    cell, c_thr = float(meta["cell"]), float(meta["c_thr"])
    base, seeds, sd = [], [], seed0
    trained = set(meta.get("seeds", [])) | set(meta.get("calibration_seeds", []))
    while len(base) < min_distinct:
        if sd not in trained:
            got = tp.build_scene(cv, torch, ctx, sd)
            if got is not None:
                base += tp.scene_pairs(ctx, *got)
                seeds.append(sd)
                _log("held-out scene seed %d: %d pairs so far" % (sd, len(base)))
        sd += 1
    cent = {}
    rng = np.random.default_rng(6)
    items, gts = [], []
    for k in range(n_items):
        A, B, T_gt = base[k % len(base)]
        if id(A) not in cent:
            cent[id(A)] = ctx.export_points(A).astype(np.float64).mean(axis=0)
        G = np.eye(4)
        G[:3, 3] = cent[id(A)]
        yaw = rng.uniform(-math.pi, math.pi)
        C = np.eye(4)
        C[:3, :3] = [[math.cos(yaw), -math.sin(yaw), 0], [math.sin(yaw), math.cos(yaw), 0], [0, 0, 1]]
        C[:3, 3] = [rng.uniform(-3, 3), rng.uniform(-3, 3), rng.uniform(-0.5, 0.5)]
        E = tp.perturbed(rng, np.eye(4), trans=0.0, yaw_deg=0.0, tilt_deg=2.0)
        items.append((A, B, G @ np.linalg.inv(C) @ np.linalg.inv(G) @ T_gt @ E))
        gts.append(T_gt)
    out = {"held_out_pairs": n_items, "distinct_pairs": len(base), "held_out_seeds": seeds, "cell_m": cell,
           "cost_threshold": c_thr, "build_s": time.perf_counter() - t0,
           "training": {k: meta[k] for k in ("pairs_train", "steps", "batch", "render_scale", "final_loss")
                        if k in meta}}
    out["training"]["scenes"] = len(meta.get("seeds", []))
    runs = {}
    out["tuning"] = ctx.autotune_align(items, 8)
    for name, fn in (("plain_8start", lambda: ctx.align_batch(items, 8)),
                     ("learned_refine", lambda: ctx.align_learned(net, items, cell, c_thr, 8)),
                     ("learned_refine_rot4", lambda: ctx.align_learned(net, items, cell, c_thr, 8, n_rot=4)),
                     ("learned_rot4_no_fallback",
                      lambda: ctx.align_learned(net, items, cell, math.inf, 8, n_rot=4))):
        fn()  # warm (buffers, registration points)
        best, res = None, None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = fn()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        T, cost, st = res
        r = {"pairs_per_s": n_items / best, "ms": best * 1e3,
             "success_1cm_0.1deg": _success(T, gts, np, 0.01, 0.1),
             "success_5cm_0.5deg": _success(T, gts, np, 0.05, 0.5)}
        r["successes_1cm"] = int(round(r["success_1cm_0.1deg"] * n_items))
        r["successes_5cm"] = int(round(r["success_5cm_0.5deg"] * n_items))
        r["aligned_per_s_1cm"] = r["pairs_per_s"] * r["success_1cm_0.1deg"]
        r["aligned_per_s_5cm"] = r["pairs_per_s"] * r["success_5cm_0.5deg"]
        if name.startswith("learned"):
            r["fallback_fraction"] = sum(1 for x in st if x["best_start"] >= 0) / n_items
        runs[name] = r
    out.update(runs)
    Tp = ctx.propose(net, items, cell, n_rot=4)
    out["proposal_only_success_0.5m_10deg"] = _success(Tp[:, 0], gts, np, 0.5, 10.0)
    out["proposal_any_of_4_turned_0.5m_10deg"] = float(np.mean(
        [any(_success([Tp[i, k]], [gts[i]], np, 0.5, 10.0) > 0 for k in range(4)) for i in range(n_items)]))
    pl, le = runs["plain_8start"], runs["learned_refine"]
    for name, key in (("learned_refine_rot4", "rot4"), ("learned_rot4_no_fallback", "rot4_no_fallback")):
        l4 = runs[name]
        for b in ("1cm", "5cm"):
            out["ratio_%s_aligned_per_s_%s" % (key, b)] = (l4["aligned_per_s_" + b] / pl["aligned_per_s_" + b]
                                                          if pl["aligned_per_s_" + b] > 0 else None)
    out["ratio_aligned_per_s_1cm"] = (le["aligned_per_s_1cm"] / pl["aligned_per_s_1cm"]
                                      if pl["aligned_per_s_1cm"] > 0 else None)
    out["ratio_aligned_per_s_5cm"] = (le["aligned_per_s_5cm"] / pl["aligned_per_s_5cm"]
                                      if pl["aligned_per_s_5cm"] > 0 else None)
    out["ratio_pairs_per_s"] = le["pairs_per_s"] / pl["pairs_per_s"]
    net.close()
    ctx.close()
    return out


def integrator_bench(cv, torch, np, w, dev, tuning, reps=2):
    """Projection mapping against raycasting (carved from the optical centre,
    and band-only rays) on the room sequence: integration-only frames/s
    (300 frames, no ESDF), TSDF+ESDF frames/s (ESDF after every frame), and
    kernel time per frame by kind."""
    out = {}
    for name, kw in (("projective", dict(integrator=cv.PROJECTIVE)),
                     ("raycast_carve", dict(integrator=cv.RAYCAST, ray_carve=1)),
                     ("raycast_band", dict(integrator=cv.RAYCAST, ray_carve=0))):
        ctx = cv.Context(voxel_size=w.voxel_size, trunc_vox=4, max_range=w.cam.max_range, d_max=w.d_max,
                         block_capacity=32768, **kw)
        ctx.set_tuning(**tuning)
        s = ctx.submap_create()
        r = {}
        for label, every in (("integrate_only", 0), ("tsdf_esdf", 1)):
            best = None
            for k in range(reps + 1):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.submap_reset(s)
                ctx.map_sequence(s, dev, w.cam.K, w.poses, esdf_every=every)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                if k > 0:  # the first pass warms up
                    best = dt if best is None else min(best, dt)
            r[label + "_frames_per_s"] = w.n_frames / best
        ctx.timing_enable(None)
        ctx.submap_reset(s)
        ctx.map_sequence(s, dev, w.cam.K, w.poses, esdf_every=0)
        r["kernel_us_per_frame"] = {k: v[0] * 1e3 / w.n_frames for k, v in ctx.timing_get().items() if v[1]}
        ctx.timing_enable([])
        info = ctx.submap_info(s)
        r["blocks"], r["voxel_updates_per_frame"] = info["n_blocks"], info["n_updates"] / w.n_frames
        out[name] = r
        ctx.close()
    p = out["projective"]["integrate_only_frames_per_s"]
    for name in ("raycast_carve", "raycast_band"):
        out[name]["integrate_only_speed_vs_projective"] = out[name]["integrate_only_frames_per_s"] / p
    return out


def esdf_modes_bench(cv, torch, np, w, dev, tuning, reps=2):
    """The exact EDT against the incremental wavefront (Sec. III-E) on the
    room sequence with an ESDF update after every frame: TSDF+ESDF frames/s,
    ESDF kernel time per update, and the wavefront's error against the exact
    field on the observed voxels of the final map."""
    out, fields = {}, {}
    for name, mode in (("exact", cv.ESDF_EXACT), ("wavefront", cv.ESDF_WAVEFRONT)):
        ctx = cv.Context(voxel_size=w.voxel_size, trunc_vox=4, max_range=w.cam.max_range, d_max=w.d_max,
                         block_capacity=32768, esdf_mode=mode)
        ctx.set_tuning(**tuning)
        s = ctx.submap_create()
        best = None
        for k in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.submap_reset(s)
            ctx.map_sequence(s, dev, w.cam.K, w.poses, esdf_every=1)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if k > 0:
                best = dt if best is None else min(best, dt)
        kinds = ["esdf_page", "esdf_sites", "edt_x", "edt_y", "edt_z", "wavefront"]
        ctx.timing_enable(kinds)
        ctx.submap_reset(s)
        ctx.map_sequence(s, dev, w.cam.K, w.poses, esdf_every=1)
        tk = ctx.timing_get()
        ctx.timing_enable([])
        out[name] = {"tsdf_esdf_frames_per_s": w.n_frames / best,
                     "esdf_kernel_us_per_update": sum(v[0] for k, v in tk.items() if k in kinds) * 1e3 / w.n_frames,
                     "launches_per_update": sum(v[1] for k, v in tk.items() if k in kinds) / w.n_frames}
        fields[name] = ctx.export_blocks(s)
        ctx.close()
    a, b = fields["exact"], fields["wavefront"]
    m = ~np.isnan(a["phi"])
    d = np.abs(a["phi"][m].astype(np.float64) - b["phi"][m])
    out["wavefront_vs_exact"] = {"observed_voxels": int(m.sum()), "equal_fraction": float((d == 0).mean()),
                                 "max_abs_m": float(d.max(initial=0)), "rms_m": float(np.sqrt((d ** 2).mean())),
                                 "same_keys": bool(np.array_equal(a["keys"], b["keys"]))}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-align", action="store_true")
    ap.add_argument("--no-mav", action="store_true")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp16"])
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay timing")
    ap.add_argument("--no-fp16", action="store_true", help="skip the FP16-storage room timing")
    ap.add_argument("--no-raycast", action="store_true", help="skip the projective / raycast comparison")
    ap.add_argument("--no-wavefront", action="store_true", help="skip the exact / wavefront ESDF comparison")
    ap.add_argument("--no-hash", action="store_true", help="skip the hash-table stress test")
    ap.add_argument("--no-copy", action="store_true", help="skip the stream-copy bandwidth measurement")
    ap.add_argument("--detail-out", default=None, help="also write the full record (JSON) to this file")
    ap.add_argument("--no-precision", action="store_true", help="skip the error statement against the binary64 oracle")
    ap.add_argument("--cfg4-align", action="store_true",
                    help="only the batched alignment of outdoor pairs from several scenes (several minutes of "
                         "rendering), printed as one JSON line")
    ap.add_argument("--mav-roofline-only", action="store_true",
                    help="outdoor workload: mapping and batched ESDF only (for counter runs)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (--gpus 1); multi-GPU runs are not supported",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import scenegen as sg
    import paper_2410_21149_amd as cv

    torch.cuda.set_device(0)
    if args.cfg4_align:
        print(json.dumps({"cfg4_align": cfg4_align_bench(cv, torch, np)}), flush=True)
        return
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    _log("generating the room workload (300 frames 640x480)")
    w = sg.room()
    frames = w.frames()
    dev = torch.from_numpy(frames).cuda()
    prec = cv.FP16 if args.precision == "fp16" else cv.FP32
    # Block capacity 2^21 (12.6 GB of D, W and phi): a captured step cannot
    # read the block count back, so the host bound grows by each frame's
    # whole frustum box (1.08 M blocks over the sequence), and updates fold
    # into the probe kernel only while that bound stays within capacity.
    ctx = cv.Context(voxel_size=w.voxel_size, trunc_vox=4, max_range=w.cam.max_range, d_max=w.d_max,
                     block_capacity=1 << 21, precision=prec)
    # a stream of its own (default priority): on the null stream the
    # pipelined step's cross-stream waits cost about a sixth of its rate
    room_stream = torch.cuda.Stream()
    ctx.set_stream(room_stream)
    torch.cuda.synchronize()  # the frames' upload (torch's stream) precedes every call
    s = ctx.submap_create()
    K = w.cam.K

    _log("census pass")
    census = run_census(ctx, s, dev, w, np)
    room_tuning = ctx.autotune_esdf([s])  # pass shapes for the full room (ESDF result unchanged)

    # which kernel dominates: one untimed step with every kernel timed
    ctx.timing_enable(None)
    ctx.submap_reset(s)
    ctx.map_sequence(s, dev, K, w.poses, esdf_every=1)
    prof = ctx.timing_get()
    ctx.timing_enable([])
    dominant = max((k for k in prof if prof[k][1] > 0), key=lambda k: prof[k][0])
    _log("per-kernel ms per step: " + ", ".join("%s %.3f" % (k, v[0]) for k, v in prof.items() if v[1]))

    def eager_step():
        ctx.submap_reset(s)
        ctx.map_sequence(s, dev, K, w.poses, esdf_every=1)

    # eager calls: the same steps issued call by call
    for _ in range(args.warmup):
        eager_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        eager_step()
    torch.cuda.synchronize()
    eager_fps = w.n_frames * args.steps / (time.perf_counter() - t0)

    # the dominant kernel's launches, bracketed by HIP events (one eager step)
    ctx.timing_enable([dominant])
    eager_step()
    torch.cuda.synchronize()
    tim = ctx.timing_get()
    ctx.timing_enable([])

    # the step captured once as a graph (reset, 300 frames, ESDF after each)
    # and replayed: W untimed replays, then K timed ones
    graph_fps = None
    if not args.no_graph:
        ctx.graph_begin()
        eager_step()
        graph = ctx.graph_end()
        for _ in range(args.warmup):
            graph.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            graph.launch()
        torch.cuda.synchronize()
        graph_fps = w.n_frames * args.steps / (time.perf_counter() - t0)
        ctx.sync()  # sticky capacity status of the replays
        graph.close()
    # value: the faster of the two ways of issuing the same step (the calls
    # one by one, or the step captured once and replayed as a graph); both
    # are reported
    if graph_fps is not None and graph_fps > eager_fps:
        fps, step_mode = graph_fps, "graph_replay"
    else:
        fps, step_mode = eager_fps, "eager"
    ms_per_step = w.n_frames / fps * 1e3

    # per-call latency: one frame integrated and its ESDF updated, then a
    # host synchronisation, frame by frame through the sequence
    lat = []
    ctx.submap_reset(s)
    torch.cuda.synchronize()
    for f in range(w.n_frames):
        t0 = time.perf_counter()
        ctx.integrate_depth(s, dev[f], K, w.poses[f])
        ctx.update_esdf(s)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    lat = np.array(lat) * 1e3
    latency = {"median_ms": float(np.median(lat)), "p99_ms": float(np.percentile(lat, 99)),
               "max_ms": float(lat.max())}

    # achievable bandwidth: a device-to-device copy of 1 GiB in this run
    copy_gbs = None
    if not args.no_copy:
        n = (1 << 30) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        best = None
        for _ in range(5):
            ev[0].record()
            dst.copy_(src)
            ev[1].record()
            torch.cuda.synchronize()
            t = ev[0].elapsed_time(ev[1])
            best = t if best is None else min(best, t)
        copy_gbs = 2 * 4 * n / (best * 1e-3) / 1e9
        del src, dst

    s_dw = 4 if prec == cv.FP16 else 8
    ms_k, n_k = tim[dominant]
    per_launch_ms = ms_k / max(n_k, 1)
    # the dominant kernel against the bytes of the unit it belongs to: one
    # ESDF update (B_esdf) or one frame's integration (B_int)
    bytes_launch = unit_bytes(dominant, census, s_dw)
    achieved = bytes_launch / (per_launch_ms * 1e-3) / 1e9
    b_int, b_esdf = frame_bytes(census, s_dw)
    kms = {k: v[0] for k, v in prof.items() if v[1]}
    roofline = {"bound": "hbm", "kernel": dominant, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dominant, room_tuning, census),
                "bytes_rule": ("B_esdf = (s_D + s_W + 4) 512 n_blocks per ESDF update" if dominant in ESDF_KINDS else
                               "B_int = 4HW + 2 (s_D + s_W) N_upd + ((s_D + s_W) 512 + 24) N_new per frame"),
                "bytes_per_launch": bytes_launch, "ms_per_launch": per_launch_ms,
                "achievable_copy_GBs": copy_gbs, "frac_achievable": (achieved / copy_gbs) if copy_gbs else None,
                # whole parts of the room step: sum of bytes over sum of kernel time
                "room_esdf": part_fraction(sum(b_esdf), sum(kms.get(k, 0.0) for k in ESDF_KINDS)),
                "room_integration": part_fraction(sum(b_int), sum(kms.get(k, 0.0) for k in INTEGRATION_KINDS))}

    result = {
        "metric": METRIC,
        "value": fps,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == cv.FP32 else "f16-storage/f32",
        "data": "synthetic",
        "config": {"workload": "room 8x6x3 m, 300 frames 640x480 fx=fy=525, 5 cm voxels, tau 4 voxels, "
                               "ESDF 2 m after every frame",
                   "frames_per_step": w.n_frames, "voxel_size": w.voxel_size, "blocks": census["n_blocks"][-1],
                   "step_mode": step_mode, "eager_frames_per_s": eager_fps,
                   "graph_replay_frames_per_s": graph_fps,
                   "voxel_updates_per_step": int(sum(census["n_upd"])),
                   "latency_per_frame": latency},
        "roofline": roofline,
        "kernel_ms_per_step": kms,
        "tuning": room_tuning,
    }
    if prec == cv.FP32 and not args.no_fp16:
        # the same steps with FP16 storage of D and W (FP32 arithmetic)
        _log("room workload with FP16 storage")
        c16 = cv.Context(voxel_size=w.voxel_size, trunc_vox=4, max_range=w.cam.max_range, d_max=w.d_max,
                         block_capacity=131072, precision=cv.FP16)
        c16.set_stream(room_stream)
        c16.set_tuning(**{k: v for k, v in room_tuning.items()})
        s16 = c16.submap_create()
        for _ in range(args.warmup):
            c16.submap_reset(s16)
            c16.map_sequence(s16, dev, K, w.poses, esdf_every=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            c16.submap_reset(s16)
            c16.map_sequence(s16, dev, K, w.poses, esdf_every=1)
        torch.cuda.synchronize()
        result["config"]["fp16_storage_frames_per_s"] = w.n_frames * args.steps / (time.perf_counter() - t0)
        c16.close()
    if prec == cv.FP32 and not args.no_raycast:
        _log("projection mapping against raycasting (room)")
        result["integrators"] = integrator_bench(cv, torch, np, w, dev, room_tuning)
    if prec == cv.FP32 and not args.no_wavefront:
        _log("exact against wavefront ESDF (room)")
        result["esdf_modes"] = esdf_modes_bench(cv, torch, np, w, dev, room_tuning)
    if not args.no_align:
        _log("alignment pairs")
        result["align"] = align_bench(cv, torch, np, w, dev)
    if not args.no_mav:
        _log("outdoor workload: 30 submaps, batched ESDF and alignment")
        result["mav"] = mav_bench(cv, torch, np, roofline_only=args.mav_roofline_only)
    if not args.no_hash:
        _log("hash-table stress test (2^26 slots, load 0.25 .. 0.85)")
        result["hash_table"] = hash_bench(cv, torch, np)
    if not args.no_precision:
        _log("precision statement (binary64 oracle)")
        result["precision"] = precision_bench(cv, torch, np, w, frames, dev)
    if not args.no_cpu_baseline:
        _log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(w, frames, args.cpu_seconds)
    ctx.close()
    detail = json.dumps(result)
    _log("bench detail: " + detail)
    if args.detail_out:
        with open(args.detail_out, "w") as fh:
            fh.write(detail + "\n")
    print(json.dumps(summary_line(result)), flush=True)


def _pick(d, *keys):
    return {k: d[k] for k in keys if isinstance(d, dict) and k in d}


def summary_line(r):
    """The one JSON line: the room step (value), the roofline of its dominant
    kernel and of the parts of the step and of the outdoor batches, the oracle
    on the host cores, and compact alignment (aligns per second and success),
    learned-proposal and precision figures.  Every figure is also in the full
    record printed to stderr."""
    line = {k: r[k] for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config") if k in r}
    roof = dict(r["roofline"])
    mav = r.get("mav", {})
    if "esdf_batch" in mav:
        e = mav["esdf_batch"]
        roof["outdoor_esdf_batch"] = dict(e["roofline"], submaps=e["submaps"], blocks=e["blocks_total"])
    if "mapping" in mav:
        m = mav["mapping"]
        roof["outdoor_mapping"] = dict(m["roofline"], frames=m["frames"], frames_per_s=m["frames_per_s"])
        if m.get("concurrent"):
            roof["outdoor_mapping_concurrent"] = _pick(m["concurrent"], "contexts", "frames_per_s", "wall_GBs",
                                                       "frac_wall")
    line["roofline"] = roof
    if "cpu_baseline" in r:
        line["cpu_baseline"] = r["cpu_baseline"]
    aligns = {}
    if "align" in r:
        a = r["align"]
        aligns["room"] = {k: _pick(a.get(k, {}), "pairs_per_s", "success") for k in ("starts_1", "starts_8")}
    if "align" in mav:
        a = mav["align"]
        aligns["outdoor"] = dict(_pick(a, "pairs", "distinct_pairs", "overlap_range"),
                                 **{k: _pick(a.get(k, {}), "pairs_per_s", "success", "success_5cm",
                                             "aligned_per_s", "median_t_err_m")
                                    for k in ("starts_1", "starts_8") if k in a})
    if aligns:
        line["aligns"] = aligns
    if "learned" in mav and "plain_8start" in mav["learned"]:
        le = mav["learned"]
        line["learned"] = dict(_pick(le, "held_out_pairs", "distinct_pairs", "held_out_seeds", "ratio_aligned_per_s_1cm",
                                     "ratio_aligned_per_s_5cm", "ratio_rot4_aligned_per_s_1cm",
                                     "ratio_rot4_aligned_per_s_5cm", "ratio_rot4_no_fallback_aligned_per_s_1cm",
                                     "ratio_rot4_no_fallback_aligned_per_s_5cm", "ratio_pairs_per_s",
                                     "proposal_only_success_0.5m_10deg", "proposal_any_of_4_turned_0.5m_10deg"),
                               **{k: _pick(le[k], "pairs_per_s", "success_1cm_0.1deg", "success_5cm_0.5deg",
                                           "successes_1cm", "successes_5cm", "fallback_fraction")
                                  for k in ("plain_8start", "learned_refine", "learned_refine_rot4",
                                            "learned_rot4_no_fallback") if k in le})
        line["learned"]["training"] = _pick(le.get("training", {}), "pairs_train", "scenes", "steps")
    if "precision" in r:
        line["precision"] = dict(r["precision"])
        if "precision" in mav.get("align", {}):
            line["precision"]["outdoor_pose"] = mav["align"]["precision"]
    return line


if __name__ == "__main__":
    main()
