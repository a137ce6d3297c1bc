"""Pins of the FP64 guiding reference (vMF mixture, reflection, MIS, samplers,
network, training loss) against closed forms, library routines and
invariants.  CPU only."""
import math

import numpy as np
import pytest
import torch
from scipy import integrate, stats

from oracle import guide_ref as G


def _rand_theta(rng, d, K, kappa_range=(0.2, 30.0)):
    mu = rng.standard_normal((K, d))
    mu /= np.linalg.norm(mu, axis=1, keepdims=True)
    kappa = np.exp(rng.uniform(np.log(kappa_range[0]), np.log(kappa_range[1]), K))
    lam = rng.dirichlet(np.ones(K))
    return mu, kappa, lam


def _circle_dirs(n):
    th = (np.arange(n) + 0.5) * 2 * np.pi / n
    return np.stack([np.cos(th), np.sin(th)], 1), 2 * np.pi / n


def _sphere_quad(n_w=400, n_phi=800):
    """Midpoint rule in (w = z, phi): exact area element dw dphi."""
    w = -1 + (np.arange(n_w) + 0.5) * 2 / n_w
    ph = (np.arange(n_phi) + 0.5) * 2 * np.pi / n_phi
    W, P = np.meshgrid(w, ph, indexing="ij")
    s = np.sqrt(1 - W ** 2)
    nu = np.stack([s * np.cos(P), s * np.sin(P), W], -1).reshape(-1, 3)
    return nu, (2 / n_w) * (2 * np.pi / n_phi)


# ----------------------------------------------------------------------------- densities

@pytest.mark.parametrize("kappa", [1e-4, 0.3, 2.0, 40.0, 3000.0])
def test_vmf2_matches_scipy_vonmises(kappa):
    th = np.linspace(-np.pi, np.pi, 101)
    nu = np.stack([np.cos(th), np.sin(th)], 1)
    mu = np.array([1.0, 0.0])
    got = np.exp(G.vmf_logpdf(nu, mu, kappa))
    ref = stats.vonmises.pdf(th, kappa)
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-300)


@pytest.mark.parametrize("kappa", [1e-4, 0.3, 2.0, 40.0, 3000.0])
def test_vmf3_normalised_closed_form(kappa):
    # density of w = mu.nu is 2 pi v(w); integrate in w
    f = lambda w: 2 * np.pi * np.exp(G.vmf_logpdf(np.array([0, 0, w]), np.array([0, 0, 1.0]), kappa))  # noqa
    cut = max(-1.0, 1.0 - 50.0 / kappa)
    val = integrate.quad(f, cut, 1, limit=400, epsabs=1e-13)[0]
    if cut > -1:
        val += integrate.quad(f, -1, cut, limit=400, epsabs=1e-13)[0]
    assert abs(val - 1) < 1e-8
    # closed form: kappa / (4 pi sinh kappa) e^{kappa w} at w = 0 (moderate kappa)
    if kappa < 50:
        v0 = np.exp(G.vmf_logpdf(np.array([1.0, 0, 0]), np.array([0, 0, 1.0]), kappa))
        assert abs(v0 - kappa / (4 * np.pi * np.sinh(kappa))) < 1e-12 * max(1, v0)


@pytest.mark.parametrize("d", [2, 3])
def test_mixture_reflected_and_mis_pdfs_normalised(d):
    rng = np.random.default_rng(10 + d)
    mu, kappa, lam = _rand_theta(rng, d, 8)
    nu, dA = _circle_dirs(20000) if d == 2 else _sphere_quad()
    assert abs(np.sum(G.mixture_pdf(nu, mu, kappa, lam)) * dA - 1) < 1e-4
    n = rng.standard_normal(d)
    n /= np.linalg.norm(n)
    pg = G.guiding_pdf(nu, mu, kappa, lam, True, n)
    assert abs(np.sum(pg) * dA - 1) < 1e-4
    assert np.all(pg[nu @ n <= 0] == 0)
    for c in (0.0, 0.37, 1.0):
        pm = G.mis_pdf(nu, mu, kappa, lam, c, d, True, n)
        assert abs(np.sum(pm) * dA - 1) < 1e-4
        pm = G.mis_pdf(nu, mu, kappa, lam, c, d)
        assert abs(np.sum(pm) * dA - 1) < 1e-4


def test_mu_perpendicular_to_wall_is_reflection_symmetric():
    """A lobe whose mean lies in the tangent plane gives V(nu) = V(nu^-)."""
    mu = np.array([[1.0, 0.0, 0.0]])
    n = np.array([0.0, 0.0, 1.0])
    rng = np.random.default_rng(0)
    nu = rng.standard_normal((100, 3))
    nu /= np.linalg.norm(nu, axis=1, keepdims=True)
    a = G.mixture_pdf(nu, mu, np.array([5.0]), np.array([1.0]))
    b = G.mixture_pdf(G.reflect(nu, n), mu, np.array([5.0]), np.array([1.0]))
    np.testing.assert_allclose(a, b, rtol=1e-13)


def test_small_kappa_single_lobe_is_uniform():
    for d in (2, 3):
        nu = np.eye(d)
        mu = np.eye(d)[:1]
        v = G.mixture_pdf(nu, mu, np.array([1e-9]), np.array([1.0]))
        np.testing.assert_allclose(v, 1 / G.sphere_area(d), rtol=1e-7)


def test_output_mapping_ranges():
    rng = np.random.default_rng(3)
    y = rng.standard_normal((50, 8 * 4 + 1)) * 5
    y[0, 2] = 50.0       # kappa' above the clamp
    mu, kappa, lam, c = G.map_outputs(y, 2, 8)
    np.testing.assert_allclose(np.linalg.norm(mu, axis=-1), 1, rtol=1e-14)
    np.testing.assert_allclose(lam.sum(-1), 1, rtol=1e-14)
    assert np.all((c > 0) & (c < 1))
    assert kappa[0, 0] == pytest.approx(math.exp(G.KAPPA_LOG_MAX))


# ----------------------------------------------------------------------------- samplers

@pytest.mark.parametrize("kappa", [5e-4, 0.5, 3.0, 60.0, 5000.0])
def test_best_fisher_ks_vs_scipy(kappa):
    rng = np.random.default_rng(int(kappa * 1000) % 997)
    n = 4000
    out = np.empty(n)
    iters = 0
    for i in range(n):
        psi, it = G.von_mises_offset(kappa, rng.random((64, 3)))
        out[i] = psi
        iters += it
    p = stats.kstest(out, stats.vonmises(kappa).cdf).pvalue
    assert p > 1e-4, p
    assert iters / n < 1.6      # Best-Fisher acceptance rate is at least 0.66


@pytest.mark.parametrize("kappa", [1e-3, 0.7, 8.0, 300.0, 8000.0])
def test_vmf3_sampler_ks_closed_form_cdf(kappa):
    rng = np.random.default_rng(int(kappa * 10) % 991)
    mu = rng.standard_normal(3)
    mu /= np.linalg.norm(mu)
    n = 4000
    nus = np.array([G.vmf3_sample(mu, kappa, rng.random(), rng.random()) for _ in range(n)])
    np.testing.assert_allclose(np.linalg.norm(nus, axis=1), 1, atol=1e-12)
    w = nus @ mu
    def cdf(t):
        # F(w) = (e^{k w} - e^{-k}) / (e^k - e^{-k}), written without overflow
        return (np.exp(kappa * (t - 1)) - np.exp(-2 * kappa)) / (1 - np.exp(-2 * kappa))
    p = stats.kstest(w, cdf).pvalue
    assert p > 1e-4, p
    # azimuth about mu is uniform
    t1, t2 = G.onb(mu)
    az = np.arctan2(nus @ t2, nus @ t1)
    ok = np.abs(w) < 0.999
    if ok.sum() > 100:
        assert stats.kstest(az[ok], stats.uniform(-np.pi, 2 * np.pi).cdf).pvalue > 1e-4


def test_onb_is_orthonormal():
    rng = np.random.default_rng(5)
    for _ in range(200):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        t1, t2 = G.onb(n)
        M = np.stack([t1, t2, n])
        np.testing.assert_allclose(M @ M.T, np.eye(3), atol=1e-12)


def test_unreflected_pdf_mass_is_von_mises_valid_half_mass():
    """Without reflection p_g on a wall is the mixture restricted to the valid
    half: its integral is sum_i lam_i P_i(valid), P_i from scipy's von Mises
    CDF; the MIS pdf integrates to 1 - c (1 - that mass), the probability that
    a draw is not wasted."""
    rng = np.random.default_rng(77)
    mu, kappa, lam = _rand_theta(rng, 2, 5, (0.3, 25.0))
    tn = 0.8
    n = np.array([math.cos(tn), math.sin(tn)])
    valid = 0.0
    for m, k, l in zip(mu, kappa, lam):
        tm = math.atan2(m[1], m[0])
        valid += l * (stats.vonmises.cdf(tn + math.pi / 2, k, loc=tm) - stats.vonmises.cdf(tn - math.pi / 2, k, loc=tm))
    def arc(f, a, b):
        return integrate.quad(lambda t: float(f(np.array([[math.cos(t), math.sin(t)]]))[0]), a, b,
                              epsabs=1e-12, epsrel=1e-12, limit=200)[0]

    pg = lambda v: G.guiding_pdf(v, mu, kappa, lam, True, n, reflected=False)
    got = arc(pg, tn - math.pi / 2, tn + math.pi / 2)
    assert got == pytest.approx(valid, abs=1e-9)
    assert arc(pg, tn + math.pi / 2, tn + 1.5 * math.pi) == 0.0
    assert valid < 0.999  # some mass lies in the wall, else the pin proves nothing
    c = 0.6
    tot = arc(lambda v: G.mis_pdf(v, mu, kappa, lam, c, 2, True, n, reflected=False), tn - math.pi / 2,
              tn + math.pi / 2)
    assert tot == pytest.approx(1 - c * (1 - valid), abs=1e-9)
    # the reflected pdf keeps all the mass
    assert arc(lambda v: G.guiding_pdf(v, mu, kappa, lam, True, n), tn - math.pi / 2,
               tn + math.pi / 2) == pytest.approx(1.0, abs=1e-9)


def test_unreflected_draws_hit_the_wall_with_the_invalid_mass():
    """The fraction of wasted draws is c times the mixture mass on the invalid
    half (2D, scipy's von Mises CDF); every non-wasted draw lies in the valid
    half and carries the MIS pdf of the unreflected mixture."""
    rng = np.random.default_rng(78)
    mu, kappa, lam = _rand_theta(rng, 2, 3, (0.5, 10.0))
    tn = -0.3
    n = np.array([math.cos(tn), math.sin(tn)])
    inval = 0.0
    for m, k, l in zip(mu, kappa, lam):
        tm = math.atan2(m[1], m[0])
        inval += l * (1 - (stats.vonmises.cdf(tn + math.pi / 2, k, loc=tm)
                           - stats.vonmises.cdf(tn - math.pi / 2, k, loc=tm)))
    c = 0.7
    N = 8000
    wall = 0
    for _ in range(N):
        nu, p, g = G.sample_direction(2, mu, kappa, lam, c, rng.random(4), rng.random(4), rng.random((64, 3)),
                                      True, n, reflected=False)
        if p == 0.0:
            wall += 1
        else:
            assert np.dot(nu, n) >= 0
            assert p == pytest.approx(G.mis_pdf(nu, mu, kappa, lam, c, 2, True, n, reflected=False), rel=1e-12)
    q = c * inval
    assert abs(wall / N - q) < 5 * math.sqrt(q * (1 - q) / N), (wall / N, q)


@pytest.mark.parametrize("d", [2, 3])
def test_mis_draw_branch_and_lobe_frequencies(d):
    rng = np.random.default_rng(20 + d)
    mu, kappa, lam = _rand_theta(rng, d, 4)
    c = 0.6
    n = 6000
    guided = 0
    lobe_counts = np.zeros(4)
    cum = np.cumsum(lam)
    for _ in range(n):
        b0 = rng.random(4)
        nu, p, g = G.sample_direction(d, mu, kappa, lam, c, b0, rng.random(4), rng.random((64, 3)))
        guided += g
        if g:
            lobe_counts[min(int(np.searchsorted(cum, b0[3] * cum[-1], side="right")), 3)] += 1
        assert p > 0
    assert abs(guided / n - c) < 5 * math.sqrt(c * (1 - c) / n)
    exp = lam * guided
    chi = np.sum((lobe_counts - exp) ** 2 / exp)
    assert stats.chi2.sf(chi, 3) > 1e-4


@pytest.mark.parametrize("d", [2, 3])
def test_c_zero_reproduces_uniform_draw(d):
    """With c = 0 the MIS draw is exactly the uniform draw from the same words."""
    rng = np.random.default_rng(1)
    mu, kappa, lam = _rand_theta(rng, d, 8)
    for _ in range(50):
        b0 = rng.random(4)
        nu, p, g = G.sample_direction(d, mu, kappa, lam, 0.0, b0, rng.random(4), rng.random((8, 3)))
        assert not g
        np.testing.assert_array_equal(nu, G.uniform_direction(d, b0[0], b0[1]))
        assert p == pytest.approx(1 / G.sphere_area(d))


# ----------------------------------------------------------------------------- mean value property

def _harmonic(d):
    if d == 2:
        return lambda p: p[..., 0] ** 3 - 3 * p[..., 0] * p[..., 1] ** 2
    return lambda p: p[..., 0] ** 2 - p[..., 1] ** 2


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("on_wall,reflected", [(False, True), (True, True), (True, False)])
def test_mean_value_property_guided_mis(d, on_wall, reflected):
    """E[ u(x + r nu) / (|S| alpha p~(nu)) ] = u(x) for harmonic u, with nu drawn
    from the MIS mixture of a random guide (reflected on a wall, alpha = 1/2;
    the wall normal is chosen so that du/dn = 0 on it, i.e. no Neumann term).
    Without reflection a guided draw into the wall scores zero, and the
    estimate must stay unbiased."""
    rng = np.random.default_rng(100 + d + 10 * on_wall + 20 * (not reflected))
    mu, kappa, lam = _rand_theta(rng, d, 8, (0.5, 20))
    c = 0.7
    u = _harmonic(d)
    if on_wall:
        # wall y = 0 with the walker above it: u_y = 0 on y = 0 for both fields
        x = np.array([0.3, 0.0] + ([0.2] if d == 3 else []))
        n = np.eye(d)[1]
        alpha = 0.5
    else:
        x = np.array([0.3, -0.2] + ([0.1] if d == 3 else []))
        n = None
        alpha = 1.0
    r = 0.5
    N = 40000
    vals = np.empty(N)
    n_wall = 0
    for i in range(N):
        nu, p, g = G.sample_direction(d, mu, kappa, lam, c, rng.random(4), rng.random(4), rng.random((64, 3)),
                                      on_wall, n, reflected)
        if p == 0.0:
            assert g and not reflected and np.dot(nu, n) <= 0
            n_wall += 1
            vals[i] = 0.0
        else:
            vals[i] = u(x + r * nu) / (G.sphere_area(d) * alpha * p)
    est, se = vals.mean(), vals.std() / math.sqrt(N)
    assert abs(est - u(x)) < 5 * se, (est, u(x), se)
    if not reflected:
        assert n_wall > 0.01 * N


# ----------------------------------------------------------------------------- network + loss

def _small_cfg(d=2):
    if d == 2:
        return G.GuideConfig(dim=2, levels=3, feats=2, log2_T=6, n_min=2, n_max=12, hidden=8, n_hidden=2, K=3,
                             aabb_lo=(-1, -1), aabb_hi=(1, 1))
    return G.GuideConfig(dim=3, levels=3, feats=2, log2_T=7, n_min=2, n_max=9, hidden=8, n_hidden=3, K=3,
                         aabb_lo=(-1, -1, -1), aabb_hi=(1, 1, 1))


def test_grid_dense_levels_reproduce_linear_functions():
    cfg = G.GuideConfig(dim=2, levels=2, feats=2, log2_T=10, n_min=4, n_max=8, aabb_lo=(-1, -1), aabb_hi=(1, 1))
    rng = np.random.default_rng(0)
    x = rng.uniform(-1, 1, size=(100, 2))
    grid = torch.zeros(cfg.L, cfg.T, cfg.F, dtype=torch.float64)
    for l in range(cfg.L):
        N = cfg.resolution(l)
        assert (N + 1) ** 2 <= cfg.T
        for i in range(N + 1):
            for j in range(N + 1):
                grid[l, i + j * (N + 1), 0] = 2.0 * i / N - 0.5 * j / N
                grid[l, i + j * (N + 1), 1] = 1.0
    f = G.encode(cfg, grid, x).numpy()
    xh = (x + 1) / 2
    for l in range(cfg.L):
        # lattice decisions are taken in float32: exact up to float32 rounding
        # of the normalised position (a wrong corner or weight errs by ~1/N)
        np.testing.assert_allclose(f[:, 2 * l], 2.0 * xh[:, 0] - 0.5 * xh[:, 1], atol=1e-6)
        np.testing.assert_allclose(f[:, 2 * l + 1], 1.0, atol=1e-12)


def test_grid_weights_partition_unity_and_hash_range():
    cfg = G.GuideConfig(dim=3, levels=4, feats=2, log2_T=8, n_min=3, n_max=40, aabb_lo=(-1,) * 3, aabb_hi=(1,) * 3)
    x = np.random.default_rng(1).uniform(-1.2, 1.2, size=(300, 3))
    for idx, w in G.grid_corners(cfg, x):
        np.testing.assert_allclose(w.sum(1), 1, rtol=1e-12)
        assert np.all(w >= 0) and idx.min() >= 0 and idx.max() < cfg.T


def _hash_kat():
    import os
    rows = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "hash_grid_kat.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                v = [int(t) for t in line.split()]
                rows[v[0]] = v[1:]
    return rows


def _check_hash_kat(primes=None, monkeypatch=None):
    if primes is not None:
        monkeypatch.setattr(G, "HASH_PRIMES", primes)
    cfg = G.GuideConfig(dim=3, levels=16, feats=2, log2_T=19, n_min=16, n_max=512, aabb_lo=(0.0,) * 3,
                        aabb_hi=(1.0,) * 3)
    assert [cfg.resolution(l) for l in range(16)] == [16, 20, 25, 32, 40, 50, 64, 80, 101, 128, 161, 203, 256,
                                                       322, 406, 512]
    out = G.grid_corners(cfg, np.array([[0.301, 0.551, 0.901]]))
    for level, want in _hash_kat().items():
        assert out[level][0][0].tolist() == want, (level, out[level][0][0].tolist(), want)


def test_hash_grid_indices_match_hand_computed_values():
    """Dense and hashed cell indices of the 3D guide's grid against values
    worked out by hand from the definitions (tests/golden/hash_grid_kat.txt)."""
    _check_hash_kat()


@pytest.mark.parametrize("primes", [(1, 2654435761, 805459863), (1, 805459861, 2654435761), (2654435761, 1, 805459861)])
def test_hash_known_answers_fail_under_a_wrong_prime(monkeypatch, primes):
    with pytest.raises(AssertionError):
        _check_hash_kat(primes, monkeypatch)


def _train_batch(cfg, rng, n=64):
    d = cfg.dim
    x = rng.uniform(-0.9, 0.9, size=(n, d))
    nu = rng.standard_normal((n, d))
    nu /= np.linalg.norm(nu, axis=1, keepdims=True)
    on = rng.random(n) < 0.4
    nrm = rng.standard_normal((n, d))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    # valid half for boundary samples
    flip = (np.sum(nu * nrm, 1) < 0) & on
    nu[flip] = nu[flip] - 2 * np.sum(nu[flip] * nrm[flip], 1, keepdims=True) * nrm[flip]
    nrm[~on] = 0
    p_sample = rng.uniform(0.05, 0.5, n)
    p_t = np.abs(rng.standard_normal(n))
    return x, nu, nrm, on, p_sample, p_t


def _init_params(cfg, rng, grid_scale=0.5):
    p = [rng.uniform(-grid_scale, grid_scale, cfg.n_grid_params)]
    for a, b in cfg.layer_shapes():
        p.append(rng.uniform(-1, 1, a * b) * math.sqrt(6 / a))
    return np.concatenate(p)


@pytest.mark.parametrize("d", [2, 3])
def test_loss_gradient_matches_central_differences(d):
    cfg = _small_cfg(d)
    rng = np.random.default_rng(7 + d)
    params = _init_params(cfg, rng)
    batch = _train_batch(cfg, rng)
    L0, g = G.loss_and_grad(cfg, params, *batch)
    # the surrogate stops the gradient of p_g inside the MIS term: freeze it at
    # its base value so that the finite differences see the same function
    pg0 = G.guiding_pdf_of_params(cfg, params, batch[0], batch[1], batch[2], batch[3])
    # MLP weights and touched grid entries
    idx = np.concatenate([rng.choice(np.arange(cfg.n_grid_params, params.size), 40, replace=False),
                          np.nonzero(g[: cfg.n_grid_params])[0][:20]])
    h = 1e-6
    for i in idx:
        pp, pm = params.copy(), params.copy()
        pp[i] += h
        pm[i] -= h
        fd = (float(G.loss(cfg, torch.tensor(pp), *batch, pg_fixed=pg0))
              - float(G.loss(cfg, torch.tensor(pm), *batch, pg_fixed=pg0))) / (2 * h)
        assert abs(fd - g[i]) <= 1e-5 * max(1.0, abs(g[i])), (i, fd, g[i])


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("reflected", [True, False])
def test_surrogate_gradients_equal_one_sample_estimators(d, reflected):
    """Autograd of the surrogate w.r.t. the mapped parameters equals the paper's
    one-sample KL gradient -p_t grad p_g / (p~ p_g) (evaluated here by central
    differences of the plain numpy pdf) and the selection-probability gradient
    -e p_t (p_g - p_u) / p~^2."""
    K = 3
    rng = np.random.default_rng(30 + d)
    n = 16
    cfg = G.GuideConfig(dim=d, K=K)
    y = rng.standard_normal((n, K * (d + 2) + 1))
    x, nu, nrm, on, p_s, p_t = _train_batch(cfg, rng, n)
    yt = torch.tensor(y, requires_grad=True)
    G.loss_per_sample(cfg, yt, nu, nrm, on, p_s, p_t, reflected=reflected).sum().backward()
    gy = yt.grad.numpy()

    def pg_of(yrow, i):
        mu, kappa, lam, c = G.map_outputs(yrow[None], d, K)
        return float(G.guiding_pdf(nu[i][None], mu[0], kappa[0], lam[0], bool(on[i]), nrm[i], reflected)[0])

    for i in range(n):
        pg = pg_of(y[i], i)
        h = 1e-6
        for j in range(K * (d + 2)):
            yp, ym = y[i].copy(), y[i].copy()
            yp[j] += h
            ym[j] -= h
            dpg = (pg_of(yp, i) - pg_of(ym, i)) / (2 * h)
            expect = -(p_t[i] / p_s[i]) * dpg / pg
            assert abs(gy[i, j] - expect) <= 1e-5 * max(1, abs(expect)), (i, j)
        c = 1 / (1 + math.exp(-y[i, -1]))
        pu = (2.0 if on[i] else 1.0) / G.sphere_area(d)
        pm = c * pg + (1 - c) * pu
        expect_c = -G.E_MIS * (p_t[i] / p_s[i]) * (pg - pu) / pm * c * (1 - c)
        assert abs(gy[i, -1] - expect_c) <= 1e-9 * max(1, abs(expect_c))
