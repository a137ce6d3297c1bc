"""Online guided walk on stars (Sec. 5.2, "Online Training Scheme").

Walks run in batches; within a batch the guide is frozen and every drawn
direction is recorded.  After the batch the tail pass turns each record into
its training target and the guide takes Adam steps on the records; the updated
guide samples the next batch.  Once ``train_until_wpp`` walks per point have
been taken, training stops and the remaining walks run inference-only in one
call.  Every walk counts toward the estimate.

All device work is issued on torch's current stream through the C ABI; the
host reads one record count per training batch.
"""
from __future__ import annotations

import dataclasses
import time

import torch

from . import api
from .guide import Guide, tail_pass


@dataclasses.dataclass
class OnlineSchedule:
    """Training schedule.  The paper trains on the first 256 of 1024 walks per
    point in batches of one walk per point over a 1024^2 grid (Sec. 5.2,
    Sec. 6.1); here the default trains on the first quarter of the walks
    (``train_fraction``) in batches of 16 walks per point, so that a batch
    over tens of thousands of points still fills the GPU and its longest walk
    does not leave most lanes idle."""
    batch_wpp: int = 16              # walks per point per training batch
    train_until_wpp: int = 0         # stop training after this many walks per point (0: use train_fraction)
    train_fraction: float = 0.25     # share of the walks that train the guide when train_until_wpp is 0
    minibatch: int = 1 << 18         # records per Adam step
    max_steps_per_batch: int = 16    # Adam steps per batch (records are subsampled beyond)
    lr: float = 1e-2
    beta1: float = 0.9
    beta2: float = 0.999
    adam_eps: float = 1e-8
    e_mis: float = 0.2
    records_per_walk: float = 64.0   # record capacity per walk (overflow is dropped and counted)


class Timer:
    """Event-based timing of phases on the current stream."""

    def __init__(self):
        self.events = {}

    def mark(self, name):
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        self.events.setdefault(name, []).append(e)

    def totals(self, pairs):
        torch.cuda.synchronize()
        out = {}
        for name, (a, b) in pairs.items():
            sa, sb = self.events.get(a, []), self.events.get(b, [])
            out[name] = sum(x.elapsed_time(y) for x, y in zip(sa, sb)) * 1e-3
        return out


def online_solve(geom, problem, pts, wpp_total, guide: Guide, schedule: OnlineSchedule = None, seed=18944,
                 acc=None, timer: Timer = None, engine="persistent"):
    """Run ``wpp_total`` walks per point with online guide training.
    ``engine`` selects the walk solver (see ``api.solve``).
    Returns (accumulator, info)."""
    sch = schedule or OnlineSchedule()
    n = pts.shape[0]
    dim = pts.shape[1]
    acc = acc if acc is not None else api.Accumulator(n, pts.device)
    timer = timer or Timer()
    until = sch.train_until_wpp if sch.train_until_wpp > 0 else int(round(sch.train_fraction * wpp_total))
    train_wpp = min(until, wpp_total)
    b = max(1, min(sch.batch_wpp, train_wpp)) if train_wpp > 0 else 0
    cap = int(n * b * sch.records_per_walk) if b else 0
    rec = api.Records(dim, cap, pts.device) if b else None
    walk_value = torch.empty(n * max(b, 1), dtype=torch.float32, device=pts.device) if b else None
    loss = torch.zeros(1, dtype=torch.float32, device=pts.device)
    info = dict(batches=0, adam_steps=0, records=0, records_dropped=0, losses=[])
    done = 0
    t0 = time.perf_counter()
    while done < train_wpp:
        w = min(b, train_wpp - done)
        rec.reset()
        timer.mark("walk0")
        api.solve(geom, problem, pts, w, seed=seed, walk_offset=done, guide=guide, acc=acc,
                  walk_value=walk_value[: n * w], records=rec, engine=engine)
        timer.mark("walk1")
        tail_pass(rec, walk_value[: n * w])
        timer.mark("tail1")
        n_rec = int(rec.count.item())
        used = min(n_rec, cap)
        info["records"] += used
        info["records_dropped"] += max(0, n_rec - cap)
        steps = min(sch.max_steps_per_batch, -(-used // sch.minibatch)) if used else 0
        stride = max(1, used // max(steps, 1))
        timer.mark("train0")
        for s in range(steps):
            begin = s * stride
            count = min(sch.minibatch, used - begin)
            guide.train_step(rec, begin, count, lr=sch.lr, beta1=sch.beta1, beta2=sch.beta2, eps=sch.adam_eps,
                             e_mis=sch.e_mis, loss_out=loss)
        timer.mark("train1")
        if steps:
            info["losses"].append(loss)
            loss = torch.zeros(1, dtype=torch.float32, device=pts.device)
        info["adam_steps"] += steps
        info["batches"] += 1
        done += w
    if done < wpp_total:
        timer.mark("walk0")
        api.solve(geom, problem, pts, wpp_total - done, seed=seed, walk_offset=done, guide=guide, acc=acc,
                  engine=engine)
        timer.mark("walk1")
    torch.cuda.synchronize()
    info["wall_s"] = time.perf_counter() - t0
    info["phase_s"] = timer.totals({"walk": ("walk0", "walk1"), "tail": ("walk1", "tail1"),
                                    "train": ("train0", "train1")})
    info["walk_launches"] = len(timer.events.get("walk0", []))
    info["losses"] = [float(x.item()) for x in info["losses"]]
    return acc, info
