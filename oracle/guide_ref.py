"""FP64 reference definitions of the guiding distribution -- TEST INFRASTRUCTURE.

Plain numpy / torch-CPU (float64) statements of what the guided sampler and its
training compute, each citing the paper passage it follows.  Shares no code
with the HIP path; the tests feed both the same seeded inputs and the same
Philox words.

Contents
* von Mises-Fisher density in 2D/3D and the K-lobe mixture (Sec. 3.3, "vmm").
* Normalization mapping of the network outputs (Sec. 4.2, Tab. "reg_map").
* Reflected guiding pdf on a Neumann boundary (Sec. 4.3), and the variant
  without reflection of the reflection ablation (Sec. 6, "Sample Reflection at
  Neumann Boundaries"): the mixture itself on the valid half, a guided draw
  into the wall scoring zero.
* Uniform directional pdf (Sec. 4.1) and the one-sample MIS pdf (Sec. 4.4,
  "mis_pdf").
* Samplers: 2D von Mises by Best & Fisher's wrapped-Cauchy rejection method;
  3D vMF by inverting the CDF of mu.nu (the paper uses a numerically stable
  vMF sampler for 3D; this is the exact inverse written from the density).
* Multi-resolution grid + MLP network (Sec. 5.2, the grid-encoding equation
  "G"), with hashed levels where a dense lattice does not fit the table.
* The training objective: the one-sample KL gradient for the mixture (Sec. 4.2,
  "one_sample_kld") and the selection-probability gradient (Sec. 4.4,
  "one_sample_sp"), expressed as a surrogate loss whose autograd gradient equals
  those two estimators.

Readings where the paper is silent: kappa' is clamped to
[KAPPA_LOG_MIN, KAPPA_LOG_MAX]; mixture output layout per lobe is
(mu'_1..mu'_d, kappa', lambda') followed by c'; the network is bias-free.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.special as sps
import torch

KAPPA_LOG_MIN = -10.0
KAPPA_LOG_MAX = 9.0
C_LOGIT = 15.0       # |c'| clamp of the selection-probability logit
E_MIS = 0.2          # fixed fraction e of the selection-probability loss (Sec. 4.4)
HASH_PRIMES = (1, 2654435761, 805459861)


def sphere_area(d):
    return 2.0 * math.pi if d == 2 else 4.0 * math.pi


# ----------------------------------------------------------------------------- vMF

def vmf_logpdf(nu, mu, kappa):
    """log v(nu | mu, kappa) on S^{d-1}; nu [..., d], mu [..., d], kappa [...].
    2D: exp(k mu.nu) / (2 pi I0(k)).  3D: k exp(k mu.nu) / (4 pi sinh k)."""
    nu = np.asarray(nu, float)
    mu = np.asarray(mu, float)
    kappa = np.asarray(kappa, float)
    d = nu.shape[-1]
    c = np.sum(nu * mu, axis=-1)
    if d == 2:
        return kappa * (c - 1.0) - np.log(2 * np.pi) - np.log(sps.i0e(kappa))
    # 3D, stable in kappa: log k - log 2pi - log(1 - e^{-2k}) + k (c - 1)
    return np.log(kappa) - np.log(2 * np.pi) - np.log(-np.expm1(-2.0 * kappa)) + kappa * (c - 1.0)


def mixture_pdf(nu, mu, kappa, lam):
    """V(nu | Theta) = sum_i lam_i v(nu | mu_i, kappa_i); mu [K, d]."""
    nu = np.asarray(nu, float)
    lp = vmf_logpdf(nu[..., None, :], mu, kappa)
    return np.sum(lam * np.exp(lp), axis=-1)


def reflect(nu, n):
    """nu^- = nu - 2 (nu.n) n  (Sec. 4.3)."""
    nu = np.asarray(nu, float)
    return nu - 2.0 * np.sum(nu * n, axis=-1, keepdims=True) * n


def guiding_pdf(nu, mu, kappa, lam, on_neumann=False, n=None, reflected=True):
    """p_g: the mixture off the Neumann boundary; on it, V(nu)+V(nu^-) on the
    valid half (nu.n > 0) and 0 elsewhere (Sec. 4.3).  Without reflection
    (``reflected=False``) it is V(nu) on the valid half: the mass V puts on the
    invalid half is the probability of a draw into the wall."""
    if not on_neumann:
        return mixture_pdf(nu, mu, kappa, lam)
    cn = np.sum(nu * n, axis=-1)
    val = mixture_pdf(nu, mu, kappa, lam)
    if reflected:
        val = val + mixture_pdf(reflect(nu, n), mu, kappa, lam)
    return np.where(cn > 0, val, 0.0)


def uniform_pdf(nu, d, on_neumann=False, n=None):
    """p_u = 1/|S^{d-1}| off the boundary, 2 H(nu.n)/|S^{d-1}| on it (Sec. 4.1)."""
    nu = np.asarray(nu, float)
    base = np.full(nu.shape[:-1], 1.0 / sphere_area(d))
    if not on_neumann:
        return base
    return np.where(np.sum(nu * n, axis=-1) > 0, 2.0 * base, 0.0)


def mis_pdf(nu, mu, kappa, lam, c, d, on_neumann=False, n=None, reflected=True):
    """p~ = c p_g + (1 - c) p_u  (Sec. 4.4, balance heuristic, one sample)."""
    return (c * guiding_pdf(nu, mu, kappa, lam, on_neumann, n, reflected)
            + (1 - c) * uniform_pdf(nu, d, on_neumann, n))


def map_outputs(y, d, K):
    """Tab. reg_map: y [..., K(d+2)+1] -> (mu [...,K,d], kappa [...,K], lam [...,K], c [...])."""
    y = np.asarray(y, float)
    lob = y[..., : K * (d + 2)].reshape(y.shape[:-1] + (K, d + 2))
    mup = lob[..., :d]
    mu = mup / np.linalg.norm(mup, axis=-1, keepdims=True)
    kappa = np.exp(np.clip(lob[..., d], KAPPA_LOG_MIN, KAPPA_LOG_MAX))
    lp = lob[..., d + 1]
    lam = np.exp(lp - lp.max(axis=-1, keepdims=True))
    lam /= lam.sum(axis=-1, keepdims=True)
    c = 1.0 / (1.0 + np.exp(-np.clip(y[..., K * (d + 2)], -C_LOGIT, C_LOGIT)))
    return mu, kappa, lam, c


# ----------------------------------------------------------------------------- samplers

def u01(words):
    """32-bit word -> uniform in [0, 1): (w >> 8) * 2^-24 (shared draw convention)."""
    return (np.asarray(words, np.uint64) >> np.uint64(8)).astype(np.float64) * 2.0 ** -24


def von_mises_offset(kappa, uniforms):
    """Best & Fisher (1979) rejection sampler for the von Mises angle offset.
    ``uniforms`` is a sequence of (U1, U2, U3) triples, one per iteration.
    Returns (psi, iterations used).  Envelope: wrapped Cauchy with parameter
    rho; any rho in (0,1) leaves the accepted law exactly von Mises."""
    k = float(kappa)
    tau = 1.0 + math.sqrt(1.0 + 4.0 * k * k)
    rho = 2.0 * k * tau / ((math.sqrt(1.0 + 4.0 * k * k) + 1.0) * (tau + math.sqrt(2.0 * tau)))
    r = (1.0 + rho * rho) / (2.0 * rho)
    for it, (u1, u2, u3) in enumerate(uniforms):
        z = math.cos(math.pi * u1)
        f = (1.0 + r * z) / (r + z)
        cc = k * (r - f)
        if cc * (2.0 - cc) > u2 or (u2 > 0 and math.log(cc / u2) + 1.0 - cc >= 0.0):
            psi = math.acos(min(1.0, max(-1.0, f)))
            return (-psi if u3 < 0.5 else psi), it + 1
    return None, len(uniforms)


def vmf3_sample(mu, kappa, eta, phi_u):
    """3D vMF by inverting F(w) = (e^{k w} - e^{-k}) / (e^k - e^{-k}) for
    w = mu.nu; azimuth uniform.  1 - w = -log1p(eta * expm1(-2k)) / k."""
    mu = np.asarray(mu, float)
    k = float(kappa)
    s = -math.log1p(eta * math.expm1(-2.0 * k)) / k
    w = 1.0 - s
    st = math.sqrt(max(0.0, s * (2.0 - s)))
    t1, t2 = onb(mu)
    ph = 2.0 * math.pi * phi_u
    return w * mu + st * (math.cos(ph) * t1 + math.sin(ph) * t2)


def onb(n):
    """Orthonormal tangent pair for a unit vector (Duff et al. 2017, branchless)."""
    sgn = math.copysign(1.0, n[2])
    a = -1.0 / (sgn + n[2])
    b = n[0] * n[1] * a
    t1 = np.array([1.0 + sgn * n[0] * n[0] * a, sgn * b, -sgn * n[0]])
    t2 = np.array([b, sgn + n[1] * n[1] * a, -n[1]])
    return t1, t2


def uniform_direction(d, u0, u1):
    if d == 2:
        th = 2.0 * math.pi * u0
        return np.array([math.cos(th), math.sin(th)])
    z = 1.0 - 2.0 * u0
    rr = math.sqrt(max(0.0, 1.0 - z * z))
    ph = 2.0 * math.pi * u1
    return np.array([rr * math.cos(ph), rr * math.sin(ph), z])


def sample_direction(d, mu, kappa, lam, c, block0, block3, bf_blocks, on_neumann=False, n=None, reflected=True):
    """One MIS draw (Sec. 4.4): with probability c pick lobe i ~ lam and draw
    from vMF(mu_i, kappa_i), else draw uniformly; on a Neumann boundary reflect
    an invalid draw about the tangent plane (Sec. 4.3).  ``block0`` = uniforms
    (dir0, dir1, mis, lobe); ``block3`` = (src_dir1, eta, phi, unused);
    ``bf_blocks`` = per-iteration (U1, U2, U3) for the 2D rejection loop.
    Returns (nu, p~(nu), guided_branch).
    With ``reflected=False`` a guided draw with nu.n <= 0 is not reflected: it
    is returned as drawn with p~ = 0, which marks a sample whose recursive term
    is zero.  Uniform draws keep using the valid half, as in plain WoSt."""
    u_dir0, u_dir1, u_mis, u_lobe = block0
    guided = u_mis < c
    if guided:
        cum = np.cumsum(lam)
        i = int(np.searchsorted(cum, u_lobe * cum[-1], side="right"))
        i = min(i, len(lam) - 1)
        if d == 2:
            psi, _ = von_mises_offset(kappa[i], bf_blocks)
            m = mu[i]
            cs, sn = math.cos(psi), math.sin(psi)
            nu = np.array([cs * m[0] - sn * m[1], sn * m[0] + cs * m[1]])
        else:
            nu = vmf3_sample(mu[i], kappa[i], block3[1], block3[2])
    else:
        nu = uniform_direction(d, u_dir0, u_dir1)
    if on_neumann:
        cn = float(np.dot(nu, n))
        if guided and not reflected and cn <= 0:
            return nu, 0.0, guided
        if cn < 0:
            nu = nu - 2.0 * cn * n
    p = mis_pdf(nu, mu, kappa, lam, c, d, on_neumann, n, reflected)
    return nu, float(p), guided


# ----------------------------------------------------------------------------- network

class GuideConfig:
    def __init__(self, dim=2, levels=8, feats=2, log2_T=16, n_min=16, n_max=1024,
                 hidden=64, n_hidden=2, K=8, aabb_lo=(-1.0, -1.0), aabb_hi=(1.0, 1.0)):
        self.dim, self.L, self.F, self.log2_T = dim, levels, feats, log2_T
        self.n_min, self.n_max, self.H, self.n_hidden, self.K = n_min, n_max, hidden, n_hidden, K
        self.lo = np.asarray(aabb_lo, float)
        self.hi = np.asarray(aabb_hi, float)

    @property
    def T(self):
        return 1 << self.log2_T

    @property
    def n_out(self):
        return self.K * (self.dim + 2) + 1

    def resolution(self, l):
        if self.L == 1:
            return self.n_min
        b = math.exp((math.log(self.n_max) - math.log(self.n_min)) / (self.L - 1))
        return int(math.floor(self.n_min * b ** l))

    def layer_shapes(self):
        shapes = [(self.L * self.F, self.H)]
        shapes += [(self.H, self.H)] * (self.n_hidden - 1)
        shapes += [(self.H, self.n_out)]
        return shapes

    @property
    def n_grid_params(self):
        return self.L * self.T * self.F

    @property
    def n_mlp_params(self):
        return sum(a * b for a, b in self.layer_shapes())


def grid_corners(cfg: GuideConfig, x):
    """Per level: integer corner indices [n, 2^d] into the level table and the
    multilinear weights [n, 2^d] (equation "G": interpolation of the embeddings
    at the corners of the enclosing cell, levels concatenated).

    The cell index is an integer decided by floating point, so the normalised
    position, cell and fractional offsets are computed in float32 with the
    same operation order as a float32 implementation would (both sides take
    that integer decision in the same precision); the weights are then used
    in float64."""
    f = np.float32
    x = np.asarray(x, float).astype(f)
    d = cfg.dim
    lo = np.asarray(cfg.lo, float).astype(f)
    inv_ext = (f(1.0) / (np.asarray(cfg.hi, float).astype(f) - lo)).astype(f)
    xh = np.minimum(np.maximum((x - lo) * inv_ext, f(0.0)), f(1.0)).astype(f)
    out = []
    for l in range(cfg.L):
        N = cfg.resolution(l)
        pos = (xh * f(N)).astype(f)
        cell = np.clip(np.floor(pos), 0, N - 1).astype(np.int64)
        fr = (pos - cell.astype(f)).astype(f).astype(np.float64)
        dense = (N + 1) ** d <= cfg.T
        idx = []
        wts = []
        for corner in range(1 << d):
            dl = [(corner >> i) & 1 for i in range(d)]
            c = cell + np.asarray(dl)
            w = np.ones(x.shape[0])
            for i in range(d):
                w = w * (fr[:, i] if dl[i] else 1.0 - fr[:, i])
            if dense:
                ix = np.zeros(x.shape[0], np.int64)
                stride = 1
                for i in range(d):
                    ix += c[:, i] * stride
                    stride *= N + 1
            else:
                hsh = np.zeros(x.shape[0], np.uint64)
                for i in range(d):
                    hsh ^= (c[:, i].astype(np.uint64) * np.uint64(HASH_PRIMES[i])) & np.uint64(0xFFFFFFFF)
                ix = (hsh & np.uint64(cfg.T - 1)).astype(np.int64)
            idx.append(ix)
            wts.append(w)
        out.append((np.stack(idx, 1), np.stack(wts, 1)))
    return out


def split_params(cfg: GuideConfig, params):
    """Flat parameter vector -> (grid [L, T, F], [W_1, ..., W_out])."""
    params = torch.as_tensor(params)
    n = cfg.n_grid_params
    grid = params[:n].reshape(cfg.L, cfg.T, cfg.F)
    Ws = []
    off = n
    for a, b in cfg.layer_shapes():
        Ws.append(params[off: off + a * b].reshape(a, b))
        off += a * b
    return grid, Ws


def encode(cfg: GuideConfig, grid, x):
    """G(x): [n, L*F] features (torch, differentiable w.r.t. grid)."""
    feats = []
    for l, (idx, w) in enumerate(grid_corners(cfg, x)):
        t = grid[l][torch.as_tensor(idx)]                 # [n, 2^d, F]
        feats.append((t * torch.as_tensor(w, dtype=t.dtype)[..., None]).sum(1))
    return torch.cat(feats, dim=1)


def _round_half(t):
    """Round to the nearest fp16 value, keeping float64 (gradient passes through)."""
    return t + (t.to(torch.float16).to(torch.float64) - t).detach()


def forward(cfg: GuideConfig, params, x, round_inputs=False):
    """NN(x | Phi): raw outputs y [n, K(d+2)+1] in float64.  With
    ``round_inputs`` every layer input (grid features, hidden activations) is
    rounded to fp16 first -- the points where a half-precision network rounds;
    the arithmetic stays float64."""
    params = torch.as_tensor(params, dtype=torch.float64)
    grid, Ws = split_params(cfg, params)
    h = encode(cfg, grid, x)
    for W in Ws[:-1]:
        if round_inputs:
            h = _round_half(h)
        h = torch.relu(h @ W)
    if round_inputs:
        h = _round_half(h)
    return h @ Ws[-1]


# ----------------------------------------------------------------------------- training loss

def _t(a):
    return torch.as_tensor(np.asarray(a, float), dtype=torch.float64)


def log_vmf_t(nu, mu, kappa, d):
    c = (nu * mu).sum(-1)
    if d == 2:
        return kappa * (c - 1.0) - math.log(2 * math.pi) - torch.log(torch.special.i0e(kappa))
    return torch.log(kappa) - math.log(2 * math.pi) - torch.log(-torch.expm1(-2.0 * kappa)) + kappa * (c - 1.0)


def loss_per_sample(cfg: GuideConfig, y, nu, n_in, on_n, p_sample, p_t, e=E_MIS, pg_fixed=None, reflected=True):
    """Surrogate whose gradients are the paper's one-sample estimators:
    l = -w [ log p_g(nu | Theta) + e log( c sg(p_g) + (1-c) p_u ) ],  w = p_t / p~_sample.
    d l / d Theta = -p_t grad p_g / (p~ p_g)        ("one_sample_kld"),
    d l / d c     = -e p_t (p_g - p_u) / p~^2        ("one_sample_sp").
    y [n, n_out] torch (requires grad), the rest numpy.  ``pg_fixed`` replaces
    sg(p_g) by given constants (for finite-difference checks of the gradient).
    ``reflected`` selects the guiding pdf on Neumann records: the reflected
    mixture (Sec. 4.3) or, without reflection, the plain mixture."""
    d, K = cfg.dim, cfg.K
    nu_t, n_t = _t(nu), _t(n_in)
    on = torch.as_tensor(np.asarray(on_n, bool))
    lob = y[:, : K * (d + 2)].reshape(-1, K, d + 2)
    mup = lob[..., :d]
    mu = mup / mup.norm(dim=-1, keepdim=True)
    kappa = torch.exp(torch.clamp(lob[..., d], KAPPA_LOG_MIN, KAPPA_LOG_MAX))
    loglam = torch.log_softmax(lob[..., d + 1], dim=-1)
    cl = torch.clamp(y[:, K * (d + 2)], -C_LOGIT, C_LOGIT)
    l1 = loglam + log_vmf_t(nu_t[:, None, :], mu, kappa, d)                       # [n, K]
    nu_r = nu_t - 2.0 * (nu_t * n_t).sum(-1, keepdim=True) * n_t
    l2 = loglam + log_vmf_t(nu_r[:, None, :], mu, kappa, d)
    both = torch.logsumexp(torch.cat([l1, l2], dim=1), dim=1)
    one = torch.logsumexp(l1, dim=1)
    log_pg = torch.where(on, both, one) if reflected else one
    area = sphere_area(d)
    pu = torch.where(on, torch.full_like(log_pg, 2.0 / area), torch.full_like(log_pg, 1.0 / area))
    log_pg_sg = log_pg.detach() if pg_fixed is None else torch.log(_t(pg_fixed))
    # log(c sg(p_g) + (1 - c) p_u) with log c = -softplus(-c'), log(1 - c) = -softplus(c')
    log_pmis = torch.logaddexp(-torch.nn.functional.softplus(-cl) + log_pg_sg,
                               -torch.nn.functional.softplus(cl) + torch.log(pu))
    w = _t(p_t) / _t(p_sample)
    return -w * (log_pg + e * log_pmis)


def loss(cfg: GuideConfig, params, x, nu, n_in, on_n, p_sample, p_t, e=E_MIS, pg_fixed=None, round_inputs=False):
    y = forward(cfg, params, x, round_inputs)
    return loss_per_sample(cfg, y, nu, n_in, on_n, p_sample, p_t, e, pg_fixed).mean()


def guiding_pdf_of_params(cfg: GuideConfig, params, x, nu, n_in, on_n):
    """p_g(nu | Theta(x)) for a batch (numpy), through the FP64 network."""
    with torch.no_grad():
        y = forward(cfg, torch.as_tensor(params, dtype=torch.float64), x).numpy()
    mu, kappa, lam, c = map_outputs(y, cfg.dim, cfg.K)
    return np.array([guiding_pdf(nu[i], mu[i], kappa[i], lam[i], bool(on_n[i]), n_in[i])
                     for i in range(len(nu))])


def loss_and_grad(cfg: GuideConfig, params, x, nu, n_in, on_n, p_sample, p_t, e=E_MIS, round_inputs=False):
    p = torch.tensor(np.asarray(params, float), dtype=torch.float64, requires_grad=True)
    L = loss(cfg, p, x, nu, n_in, on_n, p_sample, p_t, e, round_inputs=round_inputs)
    L.backward()
    return float(L.detach()), p.grad.numpy().copy()


def tail_targets(c, w, terminal_value, killed=False):
    """Reverse recursion over one walk (the training target of each step is the
    tail estimate of u at the next walk location): V_K = g (0 if killed),
    V_k = c_k + w_k V_{k+1}; returns (V_0, [|V_1|, ..., |V_K|])."""
    V = 0.0 if killed else float(terminal_value)
    tails = []
    for ck, wk in zip(reversed(list(c)), reversed(list(w))):
        tails.append(abs(V))
        V = ck + wk * V
    return V, np.asarray(tails[::-1])
