"""Benchmark: guided vs uniform walk on stars on one MI355X.

Default workload: the 3D Poisson problem at scale -- a seeded noise-displaced
sphere of 1,003,520 triangles with three spherical holes (1,018,880 triangles
in all), Neumann data on the upper half of the outer surface, Dirichlet data
x^2 - y^2 elsewhere, a source of 16 seeded Gaussian bumps, 2^20 random
interior query points.  One timed
step is one training batch of the online guided solve: 4 walks per point
(2^22 walks, guide frozen, every drawn direction recorded), the tail pass,
the batch's training set drawn from its records and the Adam steps on the
hash grid + MLP -- every stage of the hot path.  ``value`` is its walk steps
per second, end to end.

Also reported on the same line: guided vs uniform at equal time and at a
fixed relative MSE (progressive runs of both over all 2^20 points; errors on
4096 of them against a long uniform reference run), the walk kernel's
roofline position, the guide MLP's MFMA rates, and the FP64 CPU oracle timed
on a bounded sample of the same workload.  ``--workload c4`` / ``c3`` run the
same line on the 215k-triangle slice problem or the 2D mixed problem, whose
errors are taken against their closed forms.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue peak of one MI355X in lane operations: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz (a wave64 instruction occupies a SIMD for 4 cycles); the
# quoted 157.3 TFLOP/s fp32 vector peak counts a packed FMA as 4 operations
VALU_PEAK_TLANE = 256 * 64 * 2.4e9 / 1e12
# bytes read per four-wide node visit: child boxes and references, plus the
# subtree measures (Neumann sample) or normal cones (silhouettes)
NODE_BYTES = {d: {"closest_dirichlet": 16 * (2 * d + 1), "silhouette": 16 * (3 * d + 2),
                  "neumann_sample": 16 * (2 * d + 2), "neumann_visibility": 16 * (2 * d + 1),
                  "source_visibility": 16 * (2 * d + 1), "first_hit": 16 * (2 * d + 1)} for d in (2, 3)}
PRIM_BYTES = {2: {"dir": 16, "sil": 32, "neu": 32}, 3: {"dir": 48, "sil": 64, "neu": 64}}


def progress(msg):
    """A progress line on stderr (stdout carries the one JSON line)."""
    print("[bench %.0fs] %s" % (time.perf_counter() - _T0, msg), file=sys.stderr, flush=True)


_T0 = time.perf_counter()


def rel_mse(est, exact, delta=1e-2):
    return float(np.mean((est - exact) ** 2 / (exact ** 2 + delta)))


def bytes_per_step(cost, dim):
    """Algorithmic bytes per walk step: hierarchy nodes fetched and primitive
    records tested by the six queries of a step (counted by the instrumented
    kernel)."""
    nb = NODE_BYTES[dim]
    pb = PRIM_BYTES[dim]
    kinds = {"closest_dirichlet": pb["dir"], "silhouette": pb["sil"], "neumann_sample": pb["neu"],
             "neumann_visibility": pb["neu"], "source_visibility": pb["neu"], "first_hit": pb["neu"]}
    return sum(c["nodes_per_step"] * nb[q] + c["prims_per_step"] * kinds[q] for q, c in cost.items())


WALK_SOURCES = ["walk.hip", "walk_state.h", "geom_device.h", "guide_device.h", "walk_common.h", "wost_internal.h", "../build.py"]
COUNTER_PROFILES = {"c5": "walk_kernel3g_c5_counters.md", "c4": "walk_kernel3g_c4_counters.md",
                    "c3": "walk_kernel2g_c3_counters.md"}


def walk_sources_sha256():
    """Hash of the sources and build flags of the walk kernel, comments and
    blank space left out (a comment edit does not change the kernel)."""
    import hashlib
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2410_18944_amd", "csrc")
    for f in WALK_SOURCES:
        with open(os.path.join(csrc, f)) as fh:
            text = fh.read()
        if f.endswith(".py"):
            text = re.sub(r"#[^\n]*", "", text)
        else:
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            text = re.sub(r"//[^\n]*", "", text)
        h.update(re.sub(r"\s+", " ", text).strip().encode())
    return h.hexdigest()


def measured_traffic(workload):
    """Per-launch counter figures of the guided walk kernel on a workload from
    its committed rocprofv3 summary (a ``traffic-json:`` line): HBM bytes
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy), VALU instructions and
    the bound they establish; None when the summary was taken on other kernel
    sources than the ones built here."""
    path = os.path.join(ROOT, "profiles", COUNTER_PROFILES[workload])
    try:
        with open(path) as fh:
            for line in fh:
                if line.startswith("traffic-json: "):
                    rec = json.loads(line[len("traffic-json: "):])
                    if rec.get("sources_sha256") == walk_sources_sha256():
                        rec["path"] = path
                        return rec
    except OSError:
        pass
    return None


def cpu_baseline(scene, max_seconds=15.0, n_pts=64, seed=3):
    """The FP64 oracle (brute-force queries, uniform directions) on the host
    cores, on a seeded sample of the workload's points with the walks per
    point sized to about ``max_seconds`` of work."""
    import oracle
    oracle.build(force=False)
    o = oracle.OracleScene(scene)
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(scene.n_points, min(n_pts, scene.n_points), replace=False))
    pts = scene.points[idx]
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # calibrate on one walk per point, then size the sample
    t0 = time.perf_counter()
    r = o.solve(points=pts, wpp=1, nthreads=cores, point_ids=idx)
    dt = time.perf_counter() - t0
    wpp = int(np.clip(max_seconds / max(dt, 1e-6), 1, 256))
    t0 = time.perf_counter()
    r = o.solve(points=pts, wpp=wpp, nthreads=cores, point_ids=idx, walk_offset=1)
    dt = time.perf_counter() - t0
    steps = int(r["steps"].sum())
    return {"value": steps / dt, "unit": "walk steps/s", "cores": cores, "kind": "oracle",
            "sample": "%d seeded query points x %d walks = %d steps of the same workload, FP64 brute-force queries, "
                      "%.1f s" % (len(pts), wpp, steps, dt)}


MFMA_F16_PEAK = 2.5e15   # dense FP16 MFMA FLOP/s of one MI355X


def guide_mlp_rates(W, gcfg, n_train=1 << 18, n_infer=1 << 20, reps=10):
    """Standalone guide MLP throughput on MFMA: one Adam step on n_train
    records and one inference of n_infer positions, timed with HIP events on
    the launch stream.  Algorithmic FLOP: 2 P per query forward, 3 x 2 P per
    training record (forward, data and weight gradients), P = weights of the
    MLP (C3: 16 x 64 + 64 x 64 + 64 x 33 = 7,232)."""
    import torch
    g = W.Guide(gcfg, seed=3)
    d = gcfg.dim
    P = sum(a * b for a, b in [(gcfg.levels * gcfg.feats, gcfg.hidden)] + [(gcfg.hidden, gcfg.hidden)] *
            (gcfg.n_hidden - 1) + [(gcfg.hidden, gcfg.n_out)])
    rng = np.random.default_rng(9)
    lo = np.asarray(gcfg.aabb_lo[:d]); hi = np.asarray(gcfg.aabb_hi[:d])
    rec = W.Records(d, capacity=n_train)
    D = np.zeros((3 * d + 5, n_train), np.float32)
    D[0:d] = rng.uniform(lo, hi, (n_train, d)).T
    nu = rng.normal(size=(n_train, d))
    D[d:2 * d] = (nu / np.linalg.norm(nu, axis=1, keepdims=True)).T
    D[3 * d] = 1.0 / (2 * np.pi)
    D[3 * d + 4] = rng.random(n_train)
    rec.data.copy_(torch.as_tensor(D))
    rec.count.fill_(n_train)
    pts = torch.as_tensor(rng.uniform(lo, hi, (n_infer, d)), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    out = {}
    for name, fn, n, flop in (("train_step", lambda: g.train_step(rec, 0, n_train, loss_out=loss), n_train, 6 * P),
                              ("infer", lambda: g.infer(pts), n_infer, 2 * P)):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) * 1e-3 / reps
        rate = flop * n / t
        out[name] = {"n": n, "ms": round(t * 1e3, 4), "flop_per_item": flop, "tflops": round(rate / 1e12, 3),
                     "mfma_f16_frac": round(rate / MFMA_F16_PEAK, 5)}
    return out


def run_ablations(W, OnlineSchedule, online_solve, s, geom, pts, u, args, reps=2):
    """Sampling-mode ablations (number of lobes K, the selection probability
    c: 0 = uniform, 0.5 fixed, 1 = guided only, learned; sample reflection at
    Neumann points on or off) and the
    training-schedule sweep (how many walks per point train the guide, Adam
    steps per batch), each a full solve of the bench workload; mean of `reps`
    seeds.  Prints one JSON line per configuration."""
    import torch

    def one(label, sampling="mis_learned", K=8, reflect=True, c_fixed=0.5, until=args.train_until, steps=None):
        steps = steps or args.adam_steps or 16
        rows = []
        for r in range(reps):
            seed = 500 + r
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            if sampling == "uniform":
                pb = W.Problem.from_scene(s)
                e0.record()
                acc = W.solve(geom, pb, pts, args.wpp, seed=18944 + seed)
                e1.record()
                torch.cuda.synchronize()
                ph = {"walk": e0.elapsed_time(e1) * 1e-3, "train": 0.0, "tail": 0.0}
            else:
                pb = W.Problem.from_scene(s, sampling=sampling, reflect=reflect, c_fixed=c_fixed)
                g = W.Guide(W.GuideConfig.for_scene(s, K=K), seed=seed)
                g.reflect = reflect
                sched = OnlineSchedule(batch_wpp=args.batch_wpp, train_until_wpp=until, max_steps_per_batch=steps)
                e0.record()
                acc, info = online_solve(geom, pb, pts, args.wpp, g, sched, seed=18944 + seed)
                e1.record()
                torch.cuda.synchronize()
                ph = info["phase_s"]
            t = e0.elapsed_time(e1) * 1e-3
            m = acc.estimates()[0].cpu().numpy()
            st = acc.stats()
            mse = float(np.mean((m - u) ** 2))
            rows.append(dict(time_s=t, rel_mse=rel_mse(m, u), mse=mse, mse_x_time=mse * t,
                             steps_per_walk=st["steps"] / max(st["walks"], 1), walk_s=ph["walk"],
                             train_s=ph["train"], tail_s=ph["tail"]))
        out = {k: float(np.mean([r[k] for r in rows])) for k in rows[0]}
        out.update(label=label, sampling=sampling, K=K, reflect=reflect, c_fixed=c_fixed if sampling == "mis_fixed"
                   else None, train_until_wpp=until if sampling != "uniform" else 0,
                   adam_steps_per_batch=steps if sampling != "uniform" else 0, reps=reps)
        print(json.dumps(out), flush=True)

    one("uniform (c = 0)", sampling="uniform")
    one("MIS, c = 0.5 fixed", sampling="mis_fixed", c_fixed=0.5)
    one("guided only (c = 1)", sampling="guided_only")
    one("MIS, learned c (default)")
    one("learned c, no reflection", reflect=False)
    for K in (4, 16):
        one("learned c, K = %d" % K, K=K)
    for until in (128, 256):
        one("train until %d wpp" % until, until=until)
    base = args.adam_steps or 16
    for steps in (base // 2, 2 * base):
        one("%d Adam steps per batch" % steps, steps=steps)
    if args.workload == "c4":
        # training batch size at a fixed training span (Sec. 6: larger batches
        # block the walks longer)
        for b in (8, 32):
            args.batch_wpp, saved = b, args.batch_wpp
            one("batches of %d wpp" % b)
            args.batch_wpp = saved


def run_engine_ab(W, online_solve, OnlineSchedule, s, geom, pts, u, args, reps=2):
    """The persistent fused walk kernel against the multi-kernel wavefront
    solver (one kernel per stage over compacted walk queues, the paper's own
    GPU organisation; guided network inline or on a second stream) on the
    bench workload: uniform and guided online solves, same seeds; prints one
    JSON line per engine."""
    import torch

    from paper_2410_18944_amd import api

    for engine, streams in (("persistent", 1), ("wavefront", 1), ("wavefront", 2)):
        api.set_wavefront_streams(streams)
        rows = []
        for r in range(reps):
            seed = 700 + r
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            ev[0].record()
            acc_u = W.solve(geom, W.Problem.from_scene(s), pts, args.wpp, seed=18944 + seed, engine=engine)
            ev[1].record()
            g = W.Guide(W.GuideConfig.for_scene(s), seed=seed)
            sched = OnlineSchedule(batch_wpp=args.batch_wpp, train_until_wpp=args.train_until)
            ev[2].record()
            acc_g, info = online_solve(geom, W.Problem.from_scene(s, sampling="mis_learned"), pts, args.wpp, g, sched,
                                       seed=18944 + seed, engine=engine)
            ev[3].record()
            torch.cuda.synchronize()
            su, sg = acc_u.stats(), acc_g.stats()
            t_u, t_g = ev[0].elapsed_time(ev[1]) * 1e-3, ev[2].elapsed_time(ev[3]) * 1e-3
            rows.append(dict(uniform_s=t_u, uniform_steps_per_s=su["steps"] / t_u,
                             uniform_rel_mse=rel_mse(acc_u.estimates()[0].cpu().numpy(), u),
                             guided_s=t_g, guided_walk_s=info["phase_s"]["walk"],
                             guided_steps_per_s=sg["steps"] / t_g,
                             guided_rel_mse=rel_mse(acc_g.estimates()[0].cpu().numpy(), u)))
        out = {k: float(np.mean([r[k] for r in rows])) for k in rows[0]}
        out.update(engine=engine, guided_streams=streams if engine == "wavefront" else None, reps=reps,
                   wpp=args.wpp, points=int(pts.shape[0]))
        print(json.dumps(out), flush=True)
    api.set_wavefront_streams(1)


def run_lbvh(W, reps=5):
    """GPU linear-BVH build against the host build of the same closest-point
    hierarchy (the Dirichlet primitives of the two 3D workloads), and the
    closest-point query rate of both on 2^20 points; one JSON line each."""
    import torch

    import scenes
    from paper_2410_18944_amd.api import Lbvh

    for name, make in (("C4", scenes.scene_c4), ("C5", scenes.scene_c5)):
        s = make()
        dp = s.prims[s.bc == 0]
        v = np.asarray(s.verts, np.float32)
        recs = np.concatenate([v[dp[:, 0]], v[dp[:, 1]], v[dp[:, 2]], np.zeros((len(dp), 3), np.float32)], 1)
        t_recs = torch.as_tensor(recs, device="cuda").reshape(-1)
        Lbvh(3, t_recs)          # warm-up (kernel loading)
        torch.cuda.synchronize()
        tg = []
        for _ in range(reps):
            t0 = time.perf_counter()
            bv = Lbvh(3, t_recs)
            torch.cuda.synchronize()
            tg.append(time.perf_counter() - t0)
        th = []
        for _ in range(2):
            t0 = time.perf_counter()
            geo = W.Geometry(3, s.verts, dp, np.zeros(len(dp), np.uint8))
            torch.cuda.synchronize()
            th.append(time.perf_counter() - t0)
        rng = np.random.default_rng(5)
        lo, hi = s.verts.min(0), s.verts.max(0)
        q = torch.as_tensor(rng.uniform(lo, hi, (1 << 20, 3)).astype(np.float32), device="cuda")
        rates = {}
        for label, fn in (("lbvh", lambda: bv.closest(q)), ("host_bvh", lambda: geo.query(q, silhouette=False))):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(5):
                fn()
            e1.record()
            torch.cuda.synchronize()
            rates[label] = 5 * q.shape[0] / (e0.elapsed_time(e1) * 1e-3)
        print(json.dumps({"workload": name, "primitives": int(len(dp)), "lbvh_build_ms": 1e3 * min(tg),
                          "host_build_and_upload_ms": 1e3 * min(th), "lbvh_nodes": bv.n_nodes,
                          "lbvh_levels": bv.levels, "closest_queries_per_s": rates}), flush=True)


# ------------------------------------------------------------------ workloads

def setup_workload(W, name, wpp=None, points=0, batch_wpp=0, train_until=0, uniform_wpp=0):
    """Scene, geometry, query points and run settings of a workload; the
    keyword arguments override the defaults (points: a seeded subset)."""
    import torch

    import scenes
    if name == "c5":
        s = scenes.scene_c5()
        w = dict(desc="3D Poisson at scale: noise-displaced sphere, %d triangles (Neumann on the outer z > 0 half, "
                      "x^2 - y^2 Dirichlet elsewhere, 3 Dirichlet holes), source of 16 Gaussian bumps, %d random "
                      "interior points; guided: hash grid 16x2x2^19 + MLP 3x64, K=8 vMF, learned MIS, reflection; "
                      "one step = one online training batch of 4 walks/point (2^22 walks, records, tail pass, "
                      "48 Adam steps on 2^18 records)" % (s.prims.shape[0], s.n_points),
                 batch_wpp=4, train_until=16, guided_wpp=64, uniform_wpp=64, adam_steps=48, exact=None)
    elif name == "c4":
        s = scenes.scene_c4()
        w = dict(desc="3D mixed Laplace: noise-displaced sphere, %d triangles (Neumann on the outer z > 0 half, "
                      "x^2 - y^2), 3 Dirichlet holes, %d points of the 512^2 lattice on z = 0; guided: hash grid "
                      "16x2x2^19 + MLP 3x64, K=8 vMF, learned MIS, reflection; one step = one online training batch "
                      "of 16 walks/point" % (s.prims.shape[0], s.n_points),
                 batch_wpp=64, train_until=256, guided_wpp=1024, uniform_wpp=1024, adam_steps=48, compare_points=16384,
                 exact=lambda p: p[:, 0] ** 2 - p[:, 1] ** 2)
    elif name == "c3":
        s = scenes.scene_c2()
        w = dict(desc="2D mixed Laplace: 4096-segment star polygon (Neumann, Re z^3), 4 Dirichlet holes, 256x256 "
                      "lattice (%d points); guided: hash grid 8x2x2^16 + MLP 2x64, K=8 vMF, learned MIS, reflection; "
                      "one step = one online training batch of 16 walks/point" % s.n_points,
                 batch_wpp=16, train_until=64, guided_wpp=256, uniform_wpp=256, adam_steps=16,
                 exact=lambda p: p[:, 0] ** 3 - 3 * p[:, 0] * p[:, 1] ** 2)
    else:
        raise ValueError(name)
    if wpp:
        w["guided_wpp"] = w["uniform_wpp"] = wpp
    if uniform_wpp:
        w["uniform_wpp"] = uniform_wpp
    if batch_wpp:
        w["batch_wpp"] = batch_wpp
    if train_until:
        w["train_until"] = train_until
    if points and points < s.n_points:
        idx = np.sort(np.random.default_rng(1234).choice(s.n_points, points, replace=False))
        s = s.subset(idx)
        w["desc"] += "; a seeded subset of %d points" % points
    w.update(name=name, s=s, geom=W.Geometry.from_scene(s),
             pts=torch.as_tensor(s.points, dtype=torch.float32, device="cuda"),
             pb_u=W.Problem.from_scene(s), pb_g=W.Problem.from_scene(s, sampling="mis_learned"),
             gcfg=W.GuideConfig.for_scene(s))
    return w


def _interp_loglog(ts, ys, y_star):
    """Time at which a decreasing error curve (ts, ys) reaches y_star, by
    interpolation of log t against log y between the bracketing points, or
    extrapolation from the last two points (error ~ 1 / t) if never reached."""
    lt, ly = np.log(np.asarray(ts, float)), np.log(np.asarray(ys, float))
    ls = np.log(y_star)
    for i in range(1, len(ts)):
        if (ly[i - 1] - ls) * (ly[i] - ls) <= 0 and ly[i] != ly[i - 1]:
            f = (ls - ly[i - 1]) / (ly[i] - ly[i - 1])
            return float(np.exp(lt[i - 1] + f * (lt[i] - lt[i - 1])))
    if ly[-1] > ls:         # not reached: follow error ~ 1/t from the last point
        return float(np.exp(lt[-1] + (ly[-1] - ls)))
    return float(np.exp(lt[0] - (ls - ly[0])))


def _value_at(ts, ys, t_star):
    """Error at time t_star by log-log interpolation (1/t extrapolation)."""
    lt, ly = np.log(np.asarray(ts, float)), np.log(np.asarray(ys, float))
    ls = np.log(t_star)
    if ls <= lt[0]:
        return float(np.exp(ly[0] - (ls - lt[0])))
    if ls >= lt[-1]:
        return float(np.exp(ly[-1] - (ls - lt[-1])))
    return float(np.exp(np.interp(ls, lt, ly)))


def compare_guided_uniform(W, wl, seed=900, n_ref=4096, ref_wpp=2048):
    """Progressive guided (online training) and uniform solves over all the
    workload's points, with the error logged after every batch on a seeded
    subset of n_ref points: against the closed form where there is one, else
    against a uniform reference run of ref_wpp walks on the subset (its own
    variance subtracted).  Reports equal-time relMSE and the times at which
    each method reaches r* = uniform's relMSE at its last checkpoint, with
    MSE x time at r*."""
    import torch

    from paper_2410_18944_amd.driver import OnlineSchedule, OnlineSolver, Timer

    s, pts = wl["s"], wl["pts"]
    cp = wl.get("compare_points", 0)
    if cp and cp < s.n_points:
        # the comparison runs on a seeded subset of the points (the timed
        # steps use all of them)
        idx = np.sort(np.random.default_rng(seed + 5).choice(s.n_points, cp, replace=False))
        s, pts = s.subset(idx), pts[torch.as_tensor(idx, device=pts.device)]
    n = s.n_points
    rng = np.random.default_rng(seed)
    sub = np.sort(rng.choice(n, min(n_ref, n), replace=False))
    sub_t = torch.as_tensor(sub, device="cuda")
    ref_se2 = None
    if wl["exact"] is not None:
        ref = wl["exact"](s.points[sub])
        ref_note = "closed form"
    else:
        acc_r = W.solve(wl["geom"], wl["pb_u"], pts[sub_t], ref_wpp, seed=seed + 7)
        m, se, _ = acc_r.estimates()
        ref, ref_se2 = m.cpu().numpy(), (se.cpu().numpy() ** 2)
        ref_note = "uniform run of %d walks on the subset (its variance subtracted)" % ref_wpp

    def errors(sum_, sq_, cnt_):
        cnt = cnt_.double()
        mean = (sum_ / cnt).cpu().numpy()
        raw = (mean - ref) ** 2
        d2 = raw - ref_se2 if ref_se2 is not None else raw
        rel = d2 / (ref ** 2 + 1e-2)
        # the median (of the raw squared errors: never negative) is a statistic
        # that single heavy-tailed walks do not dominate
        return float(np.mean(rel)), float(np.mean(d2)), float(np.median(raw / (ref ** 2 + 1e-2)))

    def progressive(guided):
        acc = W.Accumulator(n)
        ev0 = torch.cuda.Event(enable_timing=True)
        evs, snaps, wpps = [], [], []
        b = wl["batch_wpp"]
        total = wl["guided_wpp"] if guided else wl["uniform_wpp"]
        if guided:
            g = W.Guide(wl["gcfg"], seed=seed + 1)
            sch = OnlineSchedule(batch_wpp=b, train_until_wpp=wl["train_until"],
                                 max_steps_per_batch=wl["adam_steps"])
            sol = OnlineSolver(wl["geom"], wl["pb_g"], pts, g, sch, seed=seed + 2, acc=acc, timer=Timer())
        ev0.record()
        done = 0
        while done < total:
            w = min(b, total - done)
            if guided:
                sol.batch(w, done, train=done < wl["train_until"])
            else:
                W.solve(wl["geom"], wl["pb_u"], pts, w, seed=seed + 3, walk_offset=done, acc=acc)
            done += w
            e = torch.cuda.Event(enable_timing=True)
            e.record()
            evs.append(e)
            if done % (8 * b) == 0 or done == total:
                torch.cuda.synchronize()
                progress("comparison, %s: %d of %d walks per point" % ("guided" if guided else "uniform", done, total))
            snaps.append((acc.sum[sub_t].clone(), acc.sum_sq[sub_t].clone(), acc.count[sub_t].clone()))
            wpps.append(done)
        torch.cuda.synchronize()
        ts = [ev0.elapsed_time(e) * 1e-3 for e in evs]
        errs = [errors(*sn) for sn in snaps]
        st = acc.stats()
        return dict(t=ts, rel_mse=[e[0] for e in errs], mse=[e[1] for e in errs], rel_median=[e[2] for e in errs],
                    wpp=wpps, steps_per_walk=st["steps"] / max(st["walks"], 1), steps=st["steps"])

    gu = progressive(True)
    un = progressive(False)
    r_star = un["rel_mse"][-1]
    t_u = un["t"][-1]
    t_g = _interp_loglog(gu["t"], gu["rel_mse"], r_star)
    mse_star = un["mse"][-1]
    t_eq = gu["t"][-1]
    rel_u_eq = _value_at(un["t"], un["rel_mse"], t_eq)
    out = {
        "points": int(n), "batch_wpp": wl["batch_wpp"], "adam_steps_per_batch": wl["adam_steps"],
        "error_reference": ref_note, "error_points": int(len(sub)),
        "equal_time": {"time_s": round(t_eq, 4), "rel_mse_guided": gu["rel_mse"][-1], "rel_mse_uniform": rel_u_eq,
                       "uniform_over_guided": rel_u_eq / max(gu["rel_mse"][-1], 1e-300),
                       "median_rel_err2_guided": gu["rel_median"][-1],
                       "median_rel_err2_uniform": _value_at(un["t"], un["rel_median"], t_eq)},
        "fixed_rel_mse": {"r_star": r_star, "defined_as": "uniform relMSE after %d walks/point" % wl["uniform_wpp"],
                          "t_uniform_s": round(t_u, 4), "t_guided_s": round(t_g, 4),
                          "mse_x_time_uniform": mse_star * t_u, "mse_x_time_guided": mse_star * t_g,
                          "speedup_guided_over_uniform": t_u / t_g},
        "guided": {"wpp": gu["wpp"], "t_s": [round(t, 4) for t in gu["t"]], "rel_mse": gu["rel_mse"],
                   "median_rel_err2": gu["rel_median"],
                   "steps_per_walk": gu["steps_per_walk"], "trained_through_wpp": wl["train_until"]},
        "uniform": {"wpp": un["wpp"], "t_s": [round(t, 4) for t in un["t"]], "rel_mse": un["rel_mse"],
                    "median_rel_err2": un["rel_median"],
                    "steps_per_walk": un["steps_per_walk"]},
    }
    return out


def walk_roofline(W, wl, guide, total_steps, walk_s, n_launch):
    """Roofline position of the guided walk kernel: algorithmic bytes per step
    (nodes and primitives the six queries of a step read, counted by the
    instrumented kernel on one launch of the timed shape: every point of the
    workload at the batch's walks per point, so that the per-query iteration
    overhead over a packed wave includes the end of a launch as the timed
    batches see it) against the average launch duration; the HBM bytes per
    launch measured by counters where the committed counter summary matches
    the sources built here."""
    import torch

    from paper_2410_18944_amd import api

    s, pts = wl["s"], wl["pts"]
    d = s.dim
    cost = torch.zeros(18, dtype=torch.int64, device="cuda")
    api.set_cost_counters(cost)
    a_g = W.solve(wl["geom"], wl["pb_g"], pts, wl["batch_wpp"], seed=5, guide=guide)
    torch.cuda.synchronize()
    api.set_cost_counters(None)
    cost_g = api.cost_report(cost, a_g.stats()["steps"])
    bps_g = bytes_per_step(cost_g, d)
    avg_launch = walk_s / max(n_launch, 1)
    alg_per_launch = total_steps * bps_g / max(n_launch, 1)
    achieved = alg_per_launch / max(avg_launch, 1e-12) / 1e9
    tr = measured_traffic(wl["name"])
    kern = "wost::walk_kernel%dg<false> (guided %dD walk)" % (d, d)
    out = {"kernel": kern, "bytes_per_step": round(bps_g, 1), "walk_s": round(walk_s, 4), "steps": total_steps,
           "launches": n_launch, "avg_launch_ms": round(avg_launch * 1e3, 3),
           "algorithmic_bytes_per_launch": round(alg_per_launch), "algorithmic_GBps": round(achieved, 2),
           "algorithmic_hbm_frac": round(achieved / HBM_PEAK_GBS, 4),
           "walk_sources_sha256": walk_sources_sha256()[:16],
           "nodes_per_step": {q: round(c["nodes_per_step"], 2) for q, c in cost_g.items()},
           "prims_per_step": {q: round(c["prims_per_step"], 2) for q, c in cost_g.items()},
           # wave iterations over perfectly packed ones (64 x wave iterations / lane node visits):
           # 64 / this is the mean number of lanes that advance a query per iteration
           "iterations_vs_packed": {q: round(c["divergence"], 2) for q, c in cost_g.items()}}
    if tr:
        # counter figures per launch (committed summary of the same kernel on
        # the same workload) over this run's average launch duration
        # per walk step (the profiled batch) x this run's steps per launch
        steps_per_launch = total_steps / max(n_launch, 1)
        hbm = tr["hbm_bytes_per_step"] * steps_per_launch / avg_launch / 1e9
        valu = tr["valu_insts_per_step"] * steps_per_launch * 64 / avg_launch / 1e12
        out.update({"hbm_GBps_counters": round(hbm, 1), "hbm_frac_counters": round(hbm / HBM_PEAK_GBS, 4),
                    "valu_Tlane_ops": round(valu, 3), "valu_frac": round(valu / VALU_PEAK_TLANE, 4),
                    "counter_profile": os.path.relpath(tr["path"], ROOT), "counters": tr.get("counters")})
        if tr["bound"] == "alu":
            out.update({"bound": "alu", "achieved": round(valu, 3), "peak": VALU_PEAK_TLANE, "unit": "TFLOP/s",
                        "frac": round(valu / VALU_PEAK_TLANE, 4),
                        "traffic": round(tr["hbm_bytes_per_step"] * steps_per_launch),
                        "achieved_counts": "VALU lane operations (64 per wave instruction, counted by SQ_INSTS_VALU)"})
        else:
            out.update({"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": round(tr["hbm_bytes_per_step"] * steps_per_launch)})
    else:
        out.update({"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                    "note": "no counter summary for these kernel sources: algorithmic bytes against the HBM peak"})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["c5", "c4", "c3"], default="c5")
    ap.add_argument("--wpp", type=int, default=0, help="walks per point of the comparison runs (0: workload default)")
    ap.add_argument("--batch-wpp", type=int, default=0, help="walks per point per batch (0: workload default)")
    ap.add_argument("--train-until", type=int, default=0, help="train through this many walks per point (0: default)")
    ap.add_argument("--uniform-wpp", type=int, default=0, help="walks per point of the uniform comparison run")
    ap.add_argument("--points", type=int, default=0, help="use a seeded subset of this many points (0: all)")
    ap.add_argument("--adam-steps", type=int, default=0, help="Adam steps per training batch (0: workload default)")
    ap.add_argument("--ref-points", type=int, default=4096, help="points on which the comparison measures errors")
    ap.add_argument("--ref-wpp", type=int, default=2048, help="walks per point of the reference run (no closed form)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the guided-vs-uniform comparison")
    ap.add_argument("--print-walk-sha", action="store_true", help="print the walk kernel source hash and exit")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration) and exit")
    ap.add_argument("--guide-mlp", action="store_true",
                    help="only time the standalone guide MLP (Adam step at 2^18, inference at 2^20) and exit")
    ap.add_argument("--engine-ab", action="store_true",
                    help="instead of the bench line: the persistent walk kernel against the multi-kernel "
                         "wavefront solver on the 2D workload")
    ap.add_argument("--lbvh", action="store_true",
                    help="instead of the bench line: GPU linear-BVH build and query rate against the host build")
    ap.add_argument("--ablations", action="store_true",
                    help="instead of the bench line (C2, or C4 with --workload c4): sampling-mode ablations (K, "
                         "selection c, reflection) and the "
                         "training-schedule sweep, one JSON line per configuration")
    ap.add_argument("--walk-only", action="store_true",
                    help="only the timed online batches (for profiler runs): no roofline pass, guide MLP timing, "
                         "comparison or CPU baseline")
    ap.add_argument("--compare-only", action="store_true",
                    help="only the guided-vs-uniform comparison of the workload, one JSON line")
    args = ap.parse_args()
    if args.print_walk_sha:
        print(walk_sources_sha256())
        return
    if args.copy_probe_mib > 0:
        import torch
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_mib": args.copy_probe_mib, "bytes_read_per_copy": 4 * n,
                          "bytes_written_per_copy": 4 * n, "copies": 3}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the walk-on-stars hot path here runs on a single MI355X "
              "(--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2410_18944_amd as W
    from paper_2410_18944_amd.driver import OnlineSchedule, OnlineSolver, Timer, online_solve
    import scenes

    torch.cuda.set_device(0)
    if args.lbvh:
        run_lbvh(W)
        return
    if args.ablations or args.engine_ab:
        if args.ablations and args.workload == "c4":
            # the 3D workload: a seeded subset of 16,384 of its points, 256
            # walks per point, u = x^2 - y^2 in closed form
            s = scenes.scene_c4()
            idx = np.sort(np.random.default_rng(905).choice(s.n_points, 16384, replace=False))
            s = s.subset(idx)
            u = s.points[:, 0] ** 2 - s.points[:, 1] ** 2
            args.adam_steps = args.adam_steps or 48
        else:
            s = scenes.scene_c2(wpp=256)
            u = s.points[:, 0] ** 3 - 3 * s.points[:, 0] * s.points[:, 1] ** 2
        args.wpp = args.wpp or 256
        args.batch_wpp = args.batch_wpp or 16
        args.train_until = args.train_until or 64
        pts = torch.as_tensor(s.points, dtype=torch.float32, device="cuda")
        geom = W.Geometry.from_scene(s)
        if args.ablations:
            run_ablations(W, OnlineSchedule, online_solve, s, geom, pts, u, args)
        else:
            run_engine_ab(W, online_solve, OnlineSchedule, s, geom, pts, u, args)
        return

    t_setup = time.perf_counter()
    wl = setup_workload(W, args.workload, args.wpp or None, points=args.points, batch_wpp=args.batch_wpp,
                        train_until=args.train_until, uniform_wpp=args.uniform_wpp)
    if args.adam_steps:
        wl["adam_steps"] = args.adam_steps
    s = wl["s"]
    if args.guide_mlp:
        print(json.dumps({"guide_mlp": guide_mlp_rates(W, wl["gcfg"])}))
        return
    if args.compare_only:
        print(json.dumps({"workload": args.workload, "points": s.n_points, "batch_wpp": wl["batch_wpp"],
                          "train_until": wl["train_until"], "adam_steps": wl["adam_steps"],
                          "comparison": compare_guided_uniform(W, wl, n_ref=args.ref_points, ref_wpp=args.ref_wpp)}))
        return
    setup_s = time.perf_counter() - t_setup

    # ---- the online solve whose training batches are the timed steps
    b = wl["batch_wpp"]
    g = W.Guide(wl["gcfg"], seed=1)
    sch = OnlineSchedule(batch_wpp=b, train_until_wpp=b * (args.warmup + args.steps),
                         max_steps_per_batch=wl["adam_steps"])
    timer = Timer()
    sol = OnlineSolver(wl["geom"], wl["pb_g"], wl["pts"], g, sch, seed=18944, timer=timer)
    for k in range(args.warmup):
        sol.batch(b, k * b, train=True)
    torch.cuda.synchronize()
    progress("%s: set-up and %d warm-up batches done" % (args.workload, args.warmup))
    st0 = sol.acc.stats()
    n_ev0 = len(timer.events.get("walk0", []))
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(args.warmup, args.warmup + args.steps):
        sol.batch(b, k * b, train=True)
        if (k - args.warmup) % 5 == 4:
            # the host already waits on every batch's record count, so this
            # progress line costs the timed region nothing
            progress("timed batch %d of %d" % (k - args.warmup + 1, args.steps))
    e1.record()
    torch.cuda.synchronize()
    elapsed = e0.elapsed_time(e1) * 1e-3
    wall = time.perf_counter() - t0
    st1 = sol.acc.stats()
    total_steps = st1["steps"] - st0["steps"]
    value = total_steps / elapsed
    # phase split of the timed batches (events on the launch stream)
    ph = {k: 0.0 for k in ("walk", "tail", "train")}
    pairs = {"walk": ("walk0", "walk1"), "tail": ("walk1", "tail1"), "train": ("train0", "train1")}
    for name, (a, bb) in pairs.items():
        ea, eb = timer.events.get(a, [])[n_ev0:], timer.events.get(bb, [])[n_ev0:]
        ph[name] = sum(x.elapsed_time(y) for x, y in zip(ea, eb)) * 1e-3
    info = sol.finish()
    if args.walk_only:
        print(json.dumps({"workload": args.workload, "value": round(value, 1), "unit": "walk steps/s",
                          "steps": args.steps, "walk_phase_s": ph["walk"], "avg_launch_ms": ph["walk"] / args.steps * 1e3,
                          "walk_steps": total_steps}))
        return

    progress("timed region done: %.3e walk steps/s" % value)
    roof = walk_roofline(W, wl, g, total_steps, ph["walk"], args.steps)
    mlp = guide_mlp_rates(W, wl["gcfg"])
    progress("roofline pass and guide MLP rates done")
    comp = None if args.no_compare else compare_guided_uniform(W, wl, n_ref=args.ref_points, ref_wpp=args.ref_wpp)
    if not args.no_cpu:
        progress("CPU oracle baseline")
    cpu = None if args.no_cpu else cpu_baseline(s)

    out = {
        "metric": "walk steps/s (guided WoSt, online training, end-to-end) + MSE x time guided vs uniform at fixed "
                  "relative MSE",
        "value": round(value, 1),
        "unit": "walk steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "points": s.n_points, "walks_per_step": s.n_points * b, "seed": 2410},
        "roofline": {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "cpu_baseline": cpu,
        "walk_kernel": {k: v for k, v in roof.items() if k not in ("bound", "achieved", "peak", "unit", "frac",
                                                                     "traffic")},
        "guided_step": {"walk_phase_s": round(ph["walk"] / args.steps, 4),
                        "tail_phase_s": round(ph["tail"] / args.steps, 4),
                        "train_phase_s": round(ph["train"] / args.steps, 4),
                        "adam_steps": info["adam_steps"], "records": info["records"],
                        "records_dropped": info["records_dropped"],
                        "steps_per_walk": (st1["steps"] - st0["steps"]) / max(st1["walks"] - st0["walks"], 1),
                        "walk_steps_per_s_walk_phase": round(total_steps / max(ph["walk"], 1e-9), 1)},
        "comparison": comp,
        "guide_mlp": mlp,
        "setup_s": round(setup_s, 2),
        "wall_s": round(wall, 3),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
