"""Online guided walk on stars (Sec. 5.2, "Online Training Scheme").

Walks run in batches; within a batch the guide is frozen and every drawn
direction is recorded.  After the batch the tail pass turns each record into
its training target and the guide takes Adam steps on the records; the updated
guide samples the next batch.  Once ``train_until_wpp`` walks per point have
been taken, training stops and the remaining walks run inference-only in one
call.  Every walk counts toward the estimate.

Each training batch draws its training set uniformly from all of the batch's
records, so a minibatch is not a run of records from neighbouring walks.  All
device work is issued on torch's current stream through the C ABI; the host
reads one record count per training batch.
"""
from __future__ import annotations

import dataclasses
import time

import torch

from . import api
from .guide import Guide, sample_records, tail_pass


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


class OnlineSolver:
    """One online guided solve in progress: the guide, the schedule, the
    record buffers and the per-point accumulator.  ``batch`` runs one batch of
    walks with the frozen guide; with ``train`` it also records every drawn
    direction, forms the training targets (tail pass), draws the batch's
    training set and takes the Adam steps.  All device work is issued on
    torch's current stream through the C ABI; a training batch reads one
    record count back to size its Adam steps."""

    def __init__(self, geom, problem, pts, guide: Guide, schedule: OnlineSchedule = None, seed=18944, acc=None,
                 timer: Timer = None, engine="persistent"):
        self.sch = schedule or OnlineSchedule()
        self.geom, self.problem, self.pts, self.guide = geom, problem, pts, guide
        self.seed, self.engine = seed, engine
        self.n, self.dim = pts.shape[0], pts.shape[1]
        self.acc = acc if acc is not None else api.Accumulator(self.n, pts.device)
        self.timer = timer or Timer()
        self.info = dict(batches=0, adam_steps=0, records=0, records_dropped=0, losses=[])
        self._rec = self._train = self._wv = None
        self.loss = torch.zeros(1, dtype=torch.float32, device=pts.device)

    def _buffers(self, w):
        sch = self.sch
        cap = int(self.n * w * sch.records_per_walk)
        if self._rec is None or self._rec.capacity < cap:
            self._rec = api.Records(self.dim, cap, self.pts.device)
        if self._wv is None or self._wv.numel() < self.n * w:
            self._wv = torch.empty(self.n * w, dtype=torch.float32, device=self.pts.device)
        if self._train is None:
            self._train = api.Records(self.dim, sch.max_steps_per_batch * sch.minibatch, self.pts.device)
        return self._rec, self._wv[: self.n * w], self._train

    def batch(self, w, walk_offset, train=True):
        """Walks walk_offset .. walk_offset + w - 1 of every point."""
        sch, t = self.sch, self.timer
        if not train:
            t.mark("walk0")
            api.solve(self.geom, self.problem, self.pts, w, seed=self.seed, walk_offset=walk_offset, guide=self.guide,
                      acc=self.acc, engine=self.engine)
            t.mark("walk1")
            return
        rec, wv, trs = self._buffers(w)
        rec.reset()
        t.mark("walk0")
        api.solve(self.geom, self.problem, self.pts, w, seed=self.seed, walk_offset=walk_offset, guide=self.guide,
                  acc=self.acc, walk_value=wv, records=rec, engine=self.engine)
        t.mark("walk1")
        tail_pass(rec, wv)
        t.mark("tail1")
        n_rec = int(rec.count.item())
        used = min(n_rec, rec.capacity)
        self.info["records"] += used
        self.info["records_dropped"] += max(0, n_rec - rec.capacity)
        steps = min(sch.max_steps_per_batch, -(-used // sch.minibatch)) if used else 0
        t.mark("train0")
        if steps:
            # the training set: records drawn uniformly from the whole batch,
            # so every minibatch mixes all its walks
            m = min(steps * sch.minibatch, used)
            sample_records(rec, (self.seed * 0x9E3779B97F4A7C15 + walk_offset + 1) & 0xFFFFFFFFFFFFFFFF, m, trs)
            for k in range(steps):
                begin = k * sch.minibatch
                count = min(sch.minibatch, m - begin)
                if count <= 0:
                    break
                self.guide.train_step(trs, begin, count, lr=sch.lr, beta1=sch.beta1, beta2=sch.beta2,
                                      eps=sch.adam_eps, e_mis=sch.e_mis, loss_out=self.loss)
            self.info["losses"].append(self.loss)
            self.loss = torch.zeros(1, dtype=torch.float32, device=self.pts.device)
            self.info["adam_steps"] += steps
        t.mark("train1")
        self.info["batches"] += 1

    def finish(self):
        torch.cuda.synchronize()
        info = dict(self.info)
        info["phase_s"] = self.timer.totals({"walk": ("walk0", "walk1"), "tail": ("walk1", "tail1"),
                                             "train": ("train0", "train1")})
        info["walk_launches"] = len(self.timer.events.get("walk0", []))
        info["losses"] = [float(x.item()) for x in info["losses"]]
        return info


def online_solve(geom, problem, pts, wpp_total, guide: Guide, schedule: OnlineSchedule = None, seed=18944,
                 acc=None, timer: Timer = None, engine="persistent"):
    """Run ``wpp_total`` walks per point with online guide training: batches
    of ``batch_wpp`` walks train the guide until ``train_until_wpp`` (or
    ``train_fraction`` of the walks), the rest run inference-only in one
    call.  ``engine`` selects the walk solver (see ``api.solve``).
    Returns (accumulator, info)."""
    sch = schedule or OnlineSchedule()
    until = sch.train_until_wpp if sch.train_until_wpp > 0 else int(round(sch.train_fraction * wpp_total))
    train_wpp = min(until, wpp_total)
    b = max(1, min(sch.batch_wpp, train_wpp)) if train_wpp > 0 else 0
    sol = OnlineSolver(geom, problem, pts, guide, sch, seed=seed, acc=acc, timer=timer, engine=engine)
    done = 0
    t0 = time.perf_counter()
    while done < train_wpp:
        w = min(b, train_wpp - done)
        sol.batch(w, done, train=True)
        done += w
    if done < wpp_total:
        sol.batch(wpp_total - done, done, train=False)
    info = sol.finish()
    info["wall_s"] = time.perf_counter() - t0
    return sol.acc, info
