"""Benchmark: guided vs uniform walk on stars on one MI355X.

Workload (default): the 2D mixed problem -- a seeded star-shaped 4096-segment
outer polygon with Neumann data of u = Re z^3, four circular Dirichlet holes,
the 256x256 lattice restricted to the domain (43,347 query points), 256 walks
per point.  One timed step is one guided solve of that workload with a fresh
guide trained online (batches of walks with the frozen guide and training
records, tail pass, Adam steps on the hash grid + MLP, repeated for the first
quarter of the walks, then inference-only walks), i.e. every stage of the hot
path.  ``value`` is its end-to-end walk steps per second.

Also reported on the same line: the uniform-sampling solve of the same
workload, relMSE / MSE of both against the closed form, MSE x time of both,
the walk kernel's roofline position (algorithmic bytes from instrumented
traversal counts), and the FP64 CPU oracle timed on a bounded sample.
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
# bytes read per four-wide node visit: child boxes and references, plus the
# subtree measures (Neumann sample) or normal cones (silhouettes)
NODE_BYTES = {d: {"closest_dirichlet": 16 * (2 * d + 1), "silhouette": 16 * (3 * d + 2),
                  "neumann_sample": 16 * (2 * d + 2), "neumann_visibility": 16 * (2 * d + 1),
                  "source_visibility": 16 * (2 * d + 1), "first_hit": 16 * (2 * d + 1)} for d in (2, 3)}
PRIM_BYTES = {2: {"dir": 16, "sil": 32, "neu": 32}, 3: {"dir": 48, "sil": 64, "neu": 64}}


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
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "walk_kernel2g_c3_guided_traffic.md")


def walk_sources_sha256():
    """Hash of the sources and build flags of the walk kernel."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2410_18944_amd", "csrc")
    for f in WALK_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the guided walk kernel from the committed
    FETCH_SIZE / WRITE_SIZE summary, or None when that summary was taken on
    other kernel sources than the ones built here."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            for line in fh:
                if line.startswith("traffic-json: "):
                    rec = json.loads(line[len("traffic-json: "):])
                    if rec.get("sources_sha256") == walk_sources_sha256():
                        return rec
    except OSError:
        pass
    return None


def cpu_baseline(scene, max_seconds=20.0):
    import oracle
    oracle.build(force=False)
    o = oracle.OracleScene(scene)
    idx = np.arange(0, scene.n_points, 32)
    pts = scene.points[idx]
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # calibrate on a small slice, then size the sample to about max_seconds
    t0 = time.perf_counter()
    r = o.solve(points=pts[:64], wpp=8, nthreads=cores)
    dt = time.perf_counter() - t0
    rate = r["steps"].sum() / max(dt, 1e-6)
    wpp = int(np.clip(max_seconds * rate / (len(pts) * 14.0), 4, 256))
    t0 = time.perf_counter()
    r = o.solve(points=pts, wpp=wpp, nthreads=cores)
    dt = time.perf_counter() - t0
    steps = int(r["steps"].sum())
    return {"value": steps / dt, "unit": "walk steps/s", "cores": cores, "kind": "oracle",
            "sample": "%d query points (every 32nd lattice point) x %d walks = %d steps, FP64 brute-force, %.1f s"
                      % (len(pts), wpp, steps, dt)}


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

    def one(label, sampling="mis_learned", K=8, reflect=True, c_fixed=0.5, until=args.train_until, steps=16):
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
    for steps in (8, 32):
        one("%d Adam steps per batch" % steps, steps=steps)


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--wpp", type=int, default=256)
    ap.add_argument("--batch-wpp", type=int, default=16)
    ap.add_argument("--train-until", type=int, default=64)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--print-walk-sha", action="store_true", help="print the walk kernel source hash and exit")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration) and exit")
    ap.add_argument("--guide-mlp", action="store_true",
                    help="only time the standalone guide MLP (Adam step at 2^18, inference at 2^20) and exit")
    ap.add_argument("--engine-ab", action="store_true",
                    help="instead of the bench line: the persistent walk kernel against the multi-kernel "
                         "wavefront solver on the bench workload")
    ap.add_argument("--lbvh", action="store_true",
                    help="instead of the bench line: GPU linear-BVH build and query rate against the host build")
    ap.add_argument("--ablations", action="store_true",
                    help="instead of the bench line: sampling-mode ablations (K, selection c, reflection) and the "
                         "training-schedule sweep on the same workload, one JSON line per configuration")
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
    from paper_2410_18944_amd import api
    from paper_2410_18944_amd.driver import OnlineSchedule, online_solve
    import scenes

    torch.cuda.set_device(0)
    s = scenes.scene_c2(wpp=args.wpp)
    if args.guide_mlp:
        print(json.dumps({"guide_mlp": guide_mlp_rates(W, W.GuideConfig.for_scene(s))}))
        return
    if args.lbvh:
        run_lbvh(W)
        return
    pts = torch.as_tensor(s.points, dtype=torch.float32, device="cuda")
    u = s.points[:, 0] ** 3 - 3 * s.points[:, 0] * s.points[:, 1] ** 2
    geom = W.Geometry.from_scene(s)
    pb_u = W.Problem.from_scene(s)
    pb_g = W.Problem.from_scene(s, sampling="mis_learned")
    gcfg = W.GuideConfig.for_scene(s)
    sched = OnlineSchedule(batch_wpp=args.batch_wpp, train_until_wpp=args.train_until)

    def guided_step(seed):
        g = W.Guide(gcfg, seed=seed)
        acc, info = online_solve(geom, pb_g, pts, args.wpp, g, sched, seed=18944 + seed)
        return acc, info, g

    def uniform_step(seed):
        acc = W.solve(geom, pb_u, pts, args.wpp, seed=18944 + seed)
        return acc

    for w in range(args.warmup):
        guided_step(100 + w)
        uniform_step(100 + w)
    torch.cuda.synchronize()
    if args.ablations:
        run_ablations(W, OnlineSchedule, online_solve, s, geom, pts, u, args)
        return
    if args.engine_ab:
        run_engine_ab(W, online_solve, OnlineSchedule, s, geom, pts, u, args)
        return

    # ---- timed region: K guided solves
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    total_steps = 0
    walk_s = train_s = tail_s = 0.0
    n_launch = 0
    last = None
    for k in range(args.steps):
        acc, info, g = guided_step(k + 1)
        st = acc.stats()
        total_steps += st["steps"]
        walk_s += info["phase_s"]["walk"]
        n_launch += info["walk_launches"]
        train_s += info["phase_s"]["train"]
        tail_s += info["phase_s"]["tail"]
        last = (acc, info, g)
    e1.record()
    torch.cuda.synchronize()
    elapsed = e0.elapsed_time(e1) * 1e-3
    wall = time.perf_counter() - t0
    ms_per_step = elapsed / args.steps * 1e3
    value = total_steps / elapsed

    acc_g, info_g, g_last = last
    m_g = acc_g.estimates()[0].cpu().numpy()
    st_g = acc_g.stats()
    # ---- uniform solve of the same workload (not part of `value`)
    u_e0 = torch.cuda.Event(enable_timing=True)
    u_e1 = torch.cuda.Event(enable_timing=True)
    u_e0.record()
    acc_u = uniform_step(1)
    u_e1.record()
    torch.cuda.synchronize()
    t_u = u_e0.elapsed_time(u_e1) * 1e-3
    m_u = acc_u.estimates()[0].cpu().numpy()
    st_u = acc_u.stats()
    t_g = elapsed / args.steps
    mse_g = float(np.mean((m_g - u) ** 2))
    mse_u = float(np.mean((m_u - u) ** 2))

    # ---- roofline of the walk kernel: algorithmic bytes per step from an
    # instrumented pass over a sample of the same workload
    cost = torch.zeros(18, dtype=torch.int64, device="cuda")
    api.set_cost_counters(cost)
    sample = pts[:: max(1, s.n_points // 8192)]
    a_u = W.solve(geom, pb_u, sample, 16, seed=5)
    torch.cuda.synchronize()
    bps_u = bytes_per_step(api.cost_report(cost, a_u.stats()["steps"]), 2)
    cost.zero_()
    a_g = W.solve(geom, pb_g, sample, 16, seed=5, guide=g_last)
    torch.cuda.synchronize()
    api.set_cost_counters(None)
    cost_g = api.cost_report(cost, a_g.stats()["steps"])
    bps_g = bytes_per_step(cost_g, 2)
    # dominant kernel: the guided walk kernel; time = walk phase of the timed solves
    achieved = total_steps * bps_g / max(walk_s, 1e-9) / 1e9
    tr = measured_traffic()
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": round(tr["hbm_bytes_per_launch"]) if tr else None,
                "kernel": "wost::walk_kernel2g<false> (guided 2D walk)",
                "bytes_per_step": round(bps_g, 1), "uniform_bytes_per_step": round(bps_u, 1),
                "walk_s": round(walk_s, 4), "steps": total_steps,
                "launches": n_launch, "avg_launch_ms": round(walk_s / max(n_launch, 1) * 1e3, 3),
                "algorithmic_bytes_per_launch": round(total_steps * bps_g / max(n_launch, 1)),
                "walk_sources_sha256": walk_sources_sha256()[:16]}

    mlp = guide_mlp_rates(W, gcfg)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(s)

    out = {
        "metric": "walk steps/s (guided WoSt, online training, end-to-end) + MSE x time guided vs uniform",
        "value": round(value, 1),
        "unit": "walk steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2D mixed Laplace: 4096-segment star polygon (Neumann, Re z^3), 4 Dirichlet holes, "
                               "256x256 lattice (%d points), %d walks/point, guided (hash grid 8x2x2^16 + MLP 2x64, "
                               "K=8 vMF, learned MIS, reflection), online training in %d-wpp batches for the first %d wpp"
                               % (s.n_points, args.wpp, args.batch_wpp, args.train_until),
                   "points": s.n_points, "wpp": args.wpp, "seed": 2410},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "guide_mlp": mlp,
        "guided": {"steps_per_s_end_to_end": round(value, 1), "walk_phase_s": round(walk_s / args.steps, 4),
                   "train_phase_s": round(train_s / args.steps, 4), "tail_phase_s": round(tail_s / args.steps, 4),
                   "time_s": round(t_g, 4), "rel_mse": rel_mse(m_g, u), "mse": mse_g, "mse_x_time": mse_g * t_g,
                   "adam_steps": info_g["adam_steps"], "records": info_g["records"],
                   "steps_per_walk": st_g["steps"] / max(st_g["walks"], 1)},
        "uniform": {"steps_per_s": round(st_u["steps"] / t_u, 1), "time_s": round(t_u, 4),
                    "rel_mse": rel_mse(m_u, u), "mse": mse_u, "mse_x_time": mse_u * t_u,
                    "steps_per_walk": st_u["steps"] / max(st_u["walks"], 1)},
        "mse_x_time_speedup_guided_over_uniform": (mse_u * t_u) / max(mse_g * t_g, 1e-300),
        "wall_s": round(wall, 3),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
