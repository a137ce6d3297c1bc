"""The allocation-free training step (wost_guide_train_step_noalloc) against
wost_guide_train_step: two guides in the same state take one step on the same
records, one through each entry point, and must end in the same state.  Two
calls in a row, the second on fewer records, so the library's scratch array
holds the first call's contents when the second starts.  The gradient is
summed with FP32 atomics in an unspecified order, so the comparison is to
FP32 rounding of the gradient (Adam's first and second moments), not bitwise."""
import numpy as np
import pytest
import torch

import scenes
from tests.gpu_common import say

pytestmark = pytest.mark.gpu


def _records(W, dim, n, lo, hi, seed):
    rng = np.random.default_rng(seed)
    rec = W.Records(dim, capacity=n)
    D = np.zeros((3 * dim + 5, n), np.float32)
    D[0:dim] = rng.uniform(lo, hi, (n, dim)).T
    nu = rng.normal(size=(n, dim))
    D[dim:2 * dim] = (nu / np.linalg.norm(nu, axis=1, keepdims=True)).T
    # a third of the records lie on a Neumann wall with normal +z / +y
    on = rng.random(n) < 1.0 / 3.0
    D[2 * dim + dim - 1, on] = 1.0
    D[dim + dim - 1, on] = np.abs(D[dim + dim - 1, on])
    D[3 * dim] = rng.uniform(0.05, 1.0, n)
    D[3 * dim + 4] = rng.exponential(1.0, n)
    rec.data.copy_(torch.as_tensor(D))
    rec.count.fill_(n)
    return rec


def _same_state(a, b, tol=2e-5):
    for name in ("adam_m", "adam_v"):
        x, y = getattr(a, name), getattr(b, name)
        scale = float(x.abs().max())
        err = float((x - y).abs().max())
        say("  %s: max |diff| %.3e (scale %.3e)" % (name, err, scale))
        assert scale > 0 and err <= tol * scale, (name, err, scale)


@pytest.mark.parametrize("which", ["2d", "3d"])
def test_noalloc_train_step_matches_train_step(which):
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2410_18944_amd as W
    torch.cuda.set_device(0)
    s = scenes.scene_c2() if which == "2d" else scenes.scene_cube_poisson()
    cfg = W.GuideConfig.for_scene(s)
    d = cfg.dim
    lo, hi = np.asarray(cfg.aabb_lo[:d]), np.asarray(cfg.aabb_hi[:d])
    a = W.Guide(cfg, seed=11)
    b = W.Guide(cfg, seed=11)
    assert torch.equal(a.master, b.master)
    la = torch.zeros(1, dtype=torch.float32, device="cuda")
    lb = torch.zeros(1, dtype=torch.float32, device="cuda")
    for call, n in enumerate((1 << 18, 3000)):
        rec = _records(W, d, n, lo, hi, seed=40 + call)
        say("%s call %d: %d records" % (which, call, n))
        a.train_step(rec, 0, n, loss_out=la)
        b.train_step_noalloc(rec, 0, n, loss_out=lb)
        torch.cuda.synchronize()
        fa, fb = float(la.item()), float(lb.item())
        say("  loss %.7g / %.7g" % (fa, fb))
        assert np.isfinite(fa) and abs(fa - fb) <= 1e-5 * max(abs(fa), 1e-6)
        _same_state(a, b)
        # continue both from the same state, so the next call compares one
        # step again rather than accumulated rounding
        for name in ("master", "adam_m", "adam_v"):
            getattr(b, name).copy_(getattr(a, name))
        b.sync_shadow()


def test_noalloc_rejects_oversized_call():
    """A call needing more workspace than the library's array is refused
    before any launch."""
    import paper_2410_18944_amd as W
    from paper_2410_18944_amd import _lib as L
    s = scenes.scene_cube_poisson()
    g = W.Guide(W.GuideConfig.for_scene(s), seed=1)
    n = 1 << 24
    need = int(L.load().wost_guide_train_workspace_bytes(g.h, n))
    assert need > (128 << 20)         # WOST_NOALLOC_SCRATCH_BYTES
    rec = W.Records(3, capacity=n)
    with pytest.raises(RuntimeError, match="scratch"):
        g.train_step_noalloc(rec, 0, n)
