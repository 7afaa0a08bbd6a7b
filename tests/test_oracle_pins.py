"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types an oracle formula: each checks a closed form, an
invariant, a special case that reduces to a textbook/library routine, or a
brute-force property, chosen so that a dropped term, a wrong sign, index or
exponent in the oracle fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.ndimage

from oracle import prost_oracle as O
from synth import video as V

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rng(*s):
    return np.random.default_rng(list(s))


# --------------------------------------------------------------------------
# cost functor, Sec. 3.1
# --------------------------------------------------------------------------

def test_cost_special_cases_p2_p1():
    """p = 2 makes eq. (smoothlpnorm) the shifted square r^2 + mu; p = 1 the
    Charbonnier function sqrt(r^2 + mu).  Catches a wrong exponent."""
    r = np.linspace(-3, 3, 101)
    mu = 0.37
    np.testing.assert_allclose(O.phi(r, 2.0, mu), r * r + mu, rtol=1e-15)
    np.testing.assert_allclose(O.phi(r, 1.0, mu), np.sqrt(r * r + mu), rtol=1e-15)
    np.testing.assert_allclose(O.dphi(r, 2.0, mu), 2 * r, rtol=1e-14, atol=1e-15)


def test_log_form_is_small_p_limit():
    """(2/(p mu^{p/2})) ((r^2+mu)^{p/2} - mu^{p/2}) -> log(1 + r^2/mu) as p -> 0."""
    r = np.linspace(-2, 2, 41)
    mu = 1e-3
    p = 1e-7
    lim = (2.0 / (p * mu ** (p / 2))) * (O.phi(r, p, mu) - mu ** (p / 2))
    np.testing.assert_allclose(O.phi(r, 0.0, mu, O.COST_LOG), lim, rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("form,p", [(O.COST_LP, 0.25), (O.COST_LP, 0.5), (O.COST_LP, 1.0),
                                    (O.COST_LP, 2.0), (O.COST_LOG, 0.0)])
def test_cost_derivatives_finite_differences(form, p):
    """phi' and dphi/dmu against central differences of phi."""
    r = np.linspace(-1.5, 1.5, 61) + 1e-3
    mu = 1e-2
    h = 1e-6
    fd = (O.phi(r + h, p, mu, form) - O.phi(r - h, p, mu, form)) / (2 * h)
    np.testing.assert_allclose(O.dphi(r, p, mu, form), fd, rtol=1e-7, atol=1e-9)
    hm = 1e-8
    fdm = (O.phi(r, p, mu + hm, form) - O.phi(r, p, mu - hm, form)) / (2 * hm)
    np.testing.assert_allclose(O.dphi_dmu(r, p, mu, form), fdm, rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("form,p", [(O.COST_LP, 0.25), (O.COST_LP, 0.75), (O.COST_LP, 2.0),
                                    (O.COST_LOG, 0.0)])
def test_quadratic_majoriser_brute_force(form, p):
    """phi(s) <= phi(r) + phi'(r)(s-r) + c(r)/2 (s-r)^2 for all s, with
    equality at s = r and s = -r (phi is concave in r^2 for p <= 2).  The
    equality at -r fixes c = phi'/r exactly."""
    mu = 1e-3
    s = np.linspace(-2, 2, 2001)
    for r in (-0.7, -0.03, 0.001, 0.02, 0.31, 1.4):
        q = O.phi(r, p, mu, form) + O.dphi(r, p, mu, form) * (s - r) + 0.5 * O.curv(r, p, mu, form) * (s - r) ** 2
        assert np.all(O.phi(s, p, mu, form) <= q + 1e-12 * np.maximum(1, np.abs(q)))
        q_neg = O.phi(r, p, mu, form) + O.dphi(r, p, mu, form) * (-2 * r) + 0.5 * O.curv(r, p, mu, form) * 4 * r * r
        assert abs(q_neg - O.phi(-r, p, mu, form)) <= 1e-12 * max(1.0, abs(q_neg))


@pytest.mark.parametrize("form,p", [(O.COST_LP, 0.25), (O.COST_LP, 0.5), (O.COST_LOG, 0.0)])
def test_delta_mu_coupling(form, p):
    """eq. (opt_mu): the second derivative in r vanishes at delta, and changes
    sign there (positive inside, negative outside)."""
    mu = 1e-3
    d = O.delta_from_mu(mu, p, form)
    h = 1e-7

    def d2(r):
        return (O.dphi(r + h, p, mu, form) - O.dphi(r - h, p, mu, form)) / (2 * h)

    scale = abs(d2(0.0))
    assert abs(d2(d)) < 1e-5 * scale
    assert d2(0.9 * d) > 0 > d2(1.1 * d)


def test_paper_parameters_golden():
    """Benchmark parameter set printed in Sec. 5.1, with mu from eq. (opt_mu2)."""
    g = json.load(open(os.path.join(GOLD, "paper_parameters.json")))
    assert O.mu_from_delta(g["delta"], g["p"]) == pytest.approx(g["mu_expected"], rel=1e-15)
    assert O.delta_from_mu(g["mu_expected"], g["p"]) == pytest.approx(g["delta"], rel=1e-14)
    prm = O.Params(160, 120, 3)
    assert (prm.k, prm.omega, prm.t_init, prm.t_min, prm.p, prm.cg_iters) == \
        (g["k"], g["omega"], g["t_init"], g["t_min"], g["p"], g["max_cg_steps"])


# --------------------------------------------------------------------------
# Step 1: y-solve
# --------------------------------------------------------------------------

def _problem(m=300, k=4, seed=0, frac_w=0.3):
    rng = _rng(seed)
    U = V.random_orthonormal(m, k, rng)
    x = U @ rng.standard_normal(k) * 0.3 + 0.02 * rng.standard_normal(m)
    out = rng.random(m) < 0.08
    x[out] += rng.uniform(0.2, 1.0, out.sum())
    w = np.where(rng.random(m) < frac_w, 5e-2, 1.0)
    return U, x, w


@pytest.mark.parametrize("form,p", [(O.COST_LP, 0.25), (O.COST_LOG, 0.0)])
def test_gradient_and_majoriser_along_direction(form, p):
    """g against central differences of the cost in y; and the MM bound
    f(y + a d) <= f(y) + a g.d + a^2/2 d.H d on a grid of a (brute force)."""
    U, x, w = _problem(seed=3)
    mu = 1e-3
    rng = _rng(4)
    y = rng.standard_normal(U.shape[1]) * 0.2
    g = O.grad_y(U, x, y, w, p, mu, form)
    h = 1e-6
    for j in range(U.shape[1]):
        e = np.zeros_like(y); e[j] = h
        fd = (O.cost(U, x, y + e, w, p, mu, form) - O.cost(U, x, y - e, w, p, mu, form)) / (2 * h)
        assert fd == pytest.approx(g[j], rel=1e-6, abs=1e-8)
    H = O.curvature(U, x, y, w, p, mu, form)
    f0 = O.cost(U, x, y, w, p, mu, form)
    for _ in range(5):
        d = rng.standard_normal(U.shape[1])
        for a in np.linspace(-3, 3, 121):
            q = f0 + a * g @ d + 0.5 * a * a * d @ H @ d
            assert O.cost(U, x, y + a * d, w, p, mu, form) <= q + 1e-10 * abs(q)


def test_cg_monotone_on_video():
    """The cost never increases over the CG steps of any frame."""
    wl = V.small_gray()
    sv = V.SyntheticVideo(wl.video)
    prm = O.Params(80, 60, 1, k=5, mu=wl.mu)
    st = O.initial_state(V.initial_subspace(prm.m, 5, 1), prm.P)
    for n in range(60):
        st, info = O.track_frame(st, sv.frame(n), prm)
        f = np.array(info.cg.f)
        assert np.all(np.diff(f) <= 1e-12 * f[0]), (n, f)


def test_cg_mu_infinity_is_least_squares():
    """mu -> infinity makes the cost quadratic: w = 1 gives y = U^T x; general
    w gives the weighted least-squares solution (U^T W U)^{-1} U^T W x
    (Sec. 2.1 fit)."""
    U, x, w = _problem(m=200, k=3, seed=5)
    y, _ = O.cg_solve(U, x, np.ones_like(x), np.zeros(3), 5, 0.25, 1e8)
    np.testing.assert_allclose(y, U.T @ x, rtol=1e-6)
    y, _ = O.cg_solve(U, x, w, np.zeros(3), 5, 0.25, 1e8)
    Wls = np.linalg.solve(U.T @ (U * w[:, None]), U.T @ (w * x))
    np.testing.assert_allclose(y, Wls, rtol=1e-6)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cg_p2_reaches_weighted_least_squares_in_k_steps(seed):
    """p = 2: phi is quadratic, so the CG is linear CG and ends at the exact
    weighted least-squares solution after at most k steps.  Catches a wrong
    PR+ coefficient or step length."""
    k = 5
    U, x, w = _problem(m=250, k=k, seed=10 + seed, frac_w=0.5)
    rng = _rng(seed)
    y0 = rng.standard_normal(k)
    y, rec = O.cg_solve(U, x, w, y0, k, 2.0, 0.1)
    Wls = np.linalg.solve(U.T @ (U * w[:, None]), U.T @ (w * x))
    np.testing.assert_allclose(y, Wls, rtol=1e-10, atol=1e-12)
    # w = 1: H is a multiple of I, one step is exact
    y1, _ = O.cg_solve(U, x, np.ones_like(x), y0, 1, 2.0, 0.1)
    np.testing.assert_allclose(y1, U.T @ x, rtol=1e-12, atol=1e-14)


# --------------------------------------------------------------------------
# Step 2: geodesic step
# --------------------------------------------------------------------------

def test_projection_idempotent_and_tangent():
    """eq. (gproject): pi(pi(H)) = pi(H) and U^T pi(H) = 0."""
    rng = _rng(21)
    U = V.random_orthonormal(120, 4, rng)
    Hm = rng.standard_normal((120, 3))
    P1 = O.project_tangent(U, Hm)
    np.testing.assert_allclose(O.project_tangent(U, P1), P1, atol=1e-14)
    assert np.abs(U.T @ P1).max() < 1e-14


def test_rank_one_svd_matches_lapack():
    """eq. (svd) against LAPACK's SVD of G_U = pi(eta) y^T: one nonzero
    singular value sigma = ||pi(eta)|| ||y||, singular vectors s, v up to sign."""
    U, x, w = _problem(m=150, k=4, seed=7)
    y = _rng(8).standard_normal(4)
    eta = O.eta_vector(U, x, y, w, 0.25, 1e-3)
    s, sigma, v, zeta, nu = O.rank_one_svd(U, eta, y)
    G = np.outer(O.project_tangent(U, eta), y)
    Uu, S, Vt = np.linalg.svd(G, full_matrices=False)
    assert S[0] == pytest.approx(sigma, rel=1e-13)
    assert np.all(S[1:] < 1e-12 * S[0])
    assert min(np.linalg.norm(Uu[:, 0] - s), np.linalg.norm(Uu[:, 0] + s)) < 1e-12
    assert min(np.linalg.norm(Vt[0] - v), np.linalg.norm(Vt[0] + v)) < 1e-12


def _geodesic_setup(seed=9, m=40, k=3):
    U, x, w = _problem(m=m, k=k, seed=seed)
    y = _rng(seed + 1).standard_normal(k)
    eta = O.eta_vector(U, x, y, w, 0.25, 1e-3)
    return U, x, w, y, eta


@pytest.mark.parametrize("t", [1e-4, 3e-3, 0.02])
def test_geodesic_matches_edelman_thin_svd_and_expm(t):
    """The rank-one closed form equals (i) eq. (geodesic) evaluated with the
    LAPACK thin SVD of B = -G_U and (ii) the matrix exponential of the skew
    block generator [[0, -R^T], [R, 0]] with B = Q R, on tiny inputs."""
    U, x, w, y, eta = _geodesic_setup()
    s, sigma, v, _, _ = O.rank_one_svd(U, eta, y)
    Uc = O.geodesic_rank_one(U, s, v, sigma * t)
    B = -np.outer(O.project_tangent(U, O.project_tangent(U, eta)), y)
    Th, S, Vt = np.linalg.svd(B, full_matrices=False)
    V_ = Vt.T
    Ue = (U @ V_ @ np.diag(np.cos(S * t)) + Th @ np.diag(np.sin(S * t))) @ Vt
    np.testing.assert_allclose(Uc, Ue, atol=1e-13)
    Q, R = np.linalg.qr(B)
    k = U.shape[1]
    X = np.block([[np.zeros((k, k)), -R.T], [R, np.zeros((k, k))]])
    E = scipy.linalg.expm(t * X)
    Ux = np.hstack([U, Q]) @ E[:, :k]
    np.testing.assert_allclose(Uc, Ux, atol=1e-13)


def test_geodesic_is_descent_with_rate_minus_sigma_squared():
    """d/dt h(x - U(t) y) at t = 0 equals <eta y^T, B> = -sigma^2: a
    sign error or a missing factor in the step shows here."""
    U, x, w, y, eta = _geodesic_setup(m=60, k=4)
    s, sigma, v, _, _ = O.rank_one_svd(U, eta, y)
    h = 1e-7

    def f(t):
        return O.cost(O.geodesic_rank_one(U, s, v, sigma * t), x, y, w, 0.25, 1e-3)

    slope = (f(h) - f(-h)) / (2 * h)
    assert slope == pytest.approx(-sigma ** 2, rel=1e-5)


def test_step_size_schedule():
    """Sec. 3.4: t = t_init at frame 0 and t_min from frame i_init on."""
    assert O.step_size(0, 5e-3, 1e-4, 100) == pytest.approx(5e-3, rel=1e-15)
    assert O.step_size(100, 5e-3, 1e-4, 100) == pytest.approx(1e-4, rel=1e-12)
    assert O.step_size(500, 5e-3, 1e-4, 100) == 1e-4
    assert O.step_size(50, 5e-3, 1e-4, 100) == pytest.approx(math.sqrt(5e-3 * 1e-4), rel=1e-12)


def test_orthonormality_along_trajectory():
    """The geodesic keeps U on the Stiefel manifold: ||U^T U - I|| < 1e-12
    after every frame (eq. stiefeldef)."""
    wl = V.small_gray()
    sv = V.SyntheticVideo(wl.video)
    prm = O.Params(80, 60, 1, k=5, mu=wl.mu)
    st = O.initial_state(V.initial_subspace(prm.m, 5, 1), prm.P)
    for n in range(200):
        st, _ = O.track_frame(st, sv.frame(n), prm)
        assert O.orthonormality_error(st.U) < 1e-12


@pytest.mark.parametrize("k", [2, 3])
def test_planted_subspace_recovery(k):
    """Noise- and foreground-free rank-2 video: span(U) converges to the
    planted span(Q) (principal angles < 1e-6) from a random start."""
    spec = V.VideoSpec(12, 10, 1, rank=2, seed=11, noise=0.0, fg_kind="none")
    sv = V.SyntheticVideo(spec)
    prm = O.Params(12, 10, 1, k=k, mu=1e-3, t_init=2e-3, t_min=2e-3, omega=1.0)
    st = O.initial_state(V.initial_subspace(prm.m, k, 7), prm.P)
    for n in range(3000):
        st, _ = O.track_frame(st, sv.frame(n), prm)
    assert O.principal_angles(sv.Q, st.U).max() < 1e-6


# --------------------------------------------------------------------------
# Step 3: labels and median
# --------------------------------------------------------------------------

def test_labels_recover_planted_mask_with_exact_background():
    """With U spanning the planted background and y its exact coefficients,
    noise well below delta and foreground textures far from the background,
    the labels are the planted mask; one channel alone is enough to mark a
    pixel (max over channels, Sec. 3.4)."""
    spec = V.VideoSpec(40, 30, 3, rank=3, seed=12, noise=0.001, fg_kind="rects",
                       fg_count=2, fg_density=0.1)
    sv = V.SyntheticVideo(spec)
    x, mask = sv.frame(5, with_mask=True)
    c = sv.coeffs(5)
    bg = sv.Q @ c
    far = np.abs(x - bg).reshape(3, -1).max(axis=0)
    ok = (~mask) | (far > 0.05)     # foreground pixels that differ clearly
    lab = O.pixel_labels(sv.Q, x, c, 0.02, 3)
    assert np.array_equal(lab[ok].astype(bool), mask[ok])
    # a single-channel outlier marks its pixel
    x2 = bg.copy()
    x2[2 * spec.P + 17] += 0.5
    lab2 = O.pixel_labels(sv.Q, x2, c, 0.02, 3)
    assert lab2.sum() == 1 and lab2[17] == 1


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (5, 1), (9, 13), (60, 80)])
def test_median_matches_scipy(shape):
    rng = _rng(13, *shape)
    L = (rng.random(shape) < 0.4).astype(np.uint8)
    ref = scipy.ndimage.median_filter(L, size=3, mode="nearest")
    got = O.median3x3(L.reshape(-1), *shape).reshape(shape)
    assert np.array_equal(got, ref)


def test_tracker_segments_small_video():
    """After 200 frames of the 80x60 workload the filtered mask agrees with
    the planted foreground on > 99% of pixels."""
    wl = V.small_gray()
    sv = V.SyntheticVideo(wl.video)
    prm = O.Params(80, 60, 1, k=5, mu=wl.mu)
    st = O.initial_state(V.initial_subspace(prm.m, 5, 1), prm.P)
    for n in range(200):
        st, _ = O.track_frame(st, sv.frame(n), prm)
    _, mask = sv.frame(199, with_mask=True)
    assert (st.mask.astype(bool) == mask).mean() > 0.99


# --------------------------------------------------------------------------
# precision form: re-orthonormalisation
# --------------------------------------------------------------------------

def test_lowdin_is_polar_factor():
    rng = _rng(14)
    U = V.random_orthonormal(90, 5, rng) + 1e-3 * rng.standard_normal((90, 5))
    Ul, Gp = O.lowdin(U)
    Up, Pp = scipy.linalg.polar(U)
    np.testing.assert_allclose(Ul, Up, atol=1e-13)
    np.testing.assert_allclose(Gp, Pp, atol=1e-13)
    assert O.orthonormality_error(Ul) < 1e-13


# --------------------------------------------------------------------------
# differentiable cost
# --------------------------------------------------------------------------

@pytest.mark.parametrize("form,p", [(O.COST_LP, 0.25), (O.COST_LOG, 0.0)])
def test_lpcost_backward_finite_differences(form, p):
    """All four adjoints against FP64 central differences (m=48, k=3, B=2,
    every entry)."""
    rng = _rng(15)
    m, k, B = 48, 3, 2
    U = rng.standard_normal((m, k)) * 0.3
    Y = rng.standard_normal((k, B)) * 0.3
    X = rng.standard_normal((m, B)) * 0.3
    w = np.where(rng.random(m) < 0.3, 0.1, 1.0)
    mu = 1e-2
    gout = rng.standard_normal(B)
    dX, dU, dY, dmu = O.lpcost_backward(U, Y, X, w, p, mu, gout, form)

    def L(U_, Y_, X_, mu_):
        return float(gout @ O.lpcost_forward(U_, Y_, X_, w, p, mu_, form))

    h = 1e-6
    for A, dA, name in ((U, dU, "U"), (Y, dY, "Y"), (X, dX, "X")):
        fd = np.zeros_like(A)
        for idx in np.ndindex(A.shape):
            Ap, Am = A.copy(), A.copy()
            Ap[idx] += h; Am[idx] -= h
            args_p = dict(U_=U, Y_=Y, X_=X, mu_=mu); args_m = dict(args_p)
            key = {"U": "U_", "Y": "Y_", "X": "X_"}[name]
            args_p[key] = Ap; args_m[key] = Am
            fd[idx] = (L(**args_p) - L(**args_m)) / (2 * h)
        np.testing.assert_allclose(dA, fd, rtol=1e-6, atol=1e-7)
    hm = 1e-8
    fdm = (L(U, Y, X, mu + hm) - L(U, Y, X, mu - hm)) / (2 * hm)
    assert dmu == pytest.approx(fdm, rel=1e-5)


@pytest.mark.parametrize("form,p", [(O.COST_LP, 0.25), (O.COST_LOG, 0.0)])
def test_lpcost_backward_torch_autograd(form, p):
    """Against torch's FP64 autograd of the forward written in torch ops."""
    torch = pytest.importorskip("torch")
    rng = _rng(16)
    m, k, B = 200, 4, 3
    U = rng.standard_normal((m, k)) * 0.3
    Y = rng.standard_normal((k, B)) * 0.3
    X = rng.standard_normal((m, B)) * 0.3
    w = np.where(rng.random(m) < 0.3, 0.1, 1.0)
    mu = 1e-3
    gout = rng.standard_normal(B)
    tU, tY, tX = (torch.tensor(a, requires_grad=True) for a in (U, Y, X))
    tmu = torch.tensor(mu, dtype=torch.float64, requires_grad=True)
    R = tX - tU @ tY
    if form == O.COST_LP:
        ph = (R * R + tmu) ** (p / 2)
    else:
        ph = torch.log1p(R * R / tmu)
    f = (torch.tensor(w)[:, None] * ph).sum(0)
    (f * torch.tensor(gout)).sum().backward()
    dX, dU, dY, dmu = O.lpcost_backward(U, Y, X, w, p, mu, gout, form)
    np.testing.assert_allclose(dU, tU.grad.numpy(), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(dY, tY.grad.numpy(), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(dX, tX.grad.numpy(), rtol=1e-10, atol=1e-12)
    assert dmu == pytest.approx(float(tmu.grad), rel=1e-10)
    np.testing.assert_allclose(O.lpcost_forward(U, Y, X, w, p, mu, form), f.detach().numpy(), rtol=1e-12)


# ---------------------------------------------------------------------------
# Pre-processing (Sec. 3.4, Pre- and post-processing)
# ---------------------------------------------------------------------------

def _frames(seed, n, m):
    rng = np.random.default_rng(seed)
    base = rng.random(m)
    return [base + 0.05 * rng.standard_normal(m) + 0.01 * t for t in range(n)]


def test_preprocess_statistics_match_two_pass_definitions():
    """Running average = arithmetic mean of the frames seen; the scale is the
    pooled standard deviation of the mean-subtracted entries (numpy's
    two-pass var with ddof = 1, averaged over entries) of the frames before
    the current one; frame 0 maps to exactly zero."""
    m, i_init = 50, 8
    X = _frames(3, 6, m)
    pp = O.preproc_init(m)
    for n, x in enumerate(X):
        scale_before = O.preproc_scale(pp)
        seen = np.array(X[:n])
        if n >= 2:
            assert scale_before == pytest.approx(math.sqrt(np.var(seen, axis=0, ddof=1).mean()), rel=1e-12)
        else:
            assert scale_before == 1.0
        xt, pp = O.preprocess(pp, x, n, i_init)
        seen = np.array(X[:n + 1])
        assert np.allclose(pp.mean, seen.mean(axis=0), rtol=0, atol=1e-14)
        assert np.allclose(pp.m2, ((seen - seen.mean(axis=0)) ** 2).sum(axis=0), rtol=1e-9, atol=1e-13)
        assert np.allclose(xt, (x - seen.mean(axis=0)) / scale_before, rtol=1e-12, atol=1e-13)
        if n == 0:
            assert np.array_equal(xt, np.zeros(m))


def test_preprocess_freezes_after_initialization_phase():
    m, i_init = 30, 4
    X = _frames(4, 7, m)
    pp = O.preproc_init(m)
    for n, x in enumerate(X):
        xt, pp2 = O.preprocess(pp, x, n, i_init)
        if n >= i_init:
            assert pp2.count == i_init and np.array_equal(pp2.s1, pp.s1)
            assert np.allclose(xt, (x - pp.mean) / O.preproc_scale(pp), rtol=1e-14, atol=0)
        pp = pp2


def test_preprocess_is_invariant_to_affine_intensity_changes():
    """(a x + b) for a > 0 and a constant offset per entry gives the same
    pre-processed frames once two frames are in (mean removes b, the pooled
    standard deviation absorbs a)."""
    m, i_init = 40, 10
    X = _frames(5, 5, m)
    rng = np.random.default_rng(6)
    b = rng.random(m)
    a = 3.7
    p1, p2 = O.preproc_init(m), O.preproc_init(m)
    for n, x in enumerate(X):
        x1, p1 = O.preprocess(p1, x, n, i_init)
        x2, p2 = O.preprocess(p2, a * x + b, n, i_init)
        if n >= 2:
            assert np.allclose(x1, x2, rtol=1e-9, atol=1e-11)


def test_tracker_with_preprocessing_on_static_scene_stays_still():
    """A static background with noise: after pre-processing the frames are
    zero-mean noise of unit scale, the tracker runs on them and state keeps
    its shape; frame 0 (all zero after mean removal) changes nothing."""
    prm = O.Params(12, 10, 1, k=2, preprocess=True, i_init=5)
    rng = np.random.default_rng(7)
    st = O.initial_state(V.initial_subspace(prm.m, 2, 8), prm.P)
    bg = rng.random(prm.m)
    st1, info = O.track_frame(st, bg + 0.01 * rng.standard_normal(prm.m), prm)
    assert np.array_equal(info.x, np.zeros(prm.m))
    assert np.array_equal(st1.U, st.U) and not info.updated
    assert st1.pre.count == 1
    for n in range(1, 8):
        st1, info = O.track_frame(st1, bg + 0.01 * rng.standard_normal(prm.m), prm)
    assert st1.pre.count == 5
    assert abs(np.std(info.x) - 1.0) < 0.5


# ---------------------------------------------------------------------------
# Segmentation quality measures (Sec. 5) and the delta sweep
# ---------------------------------------------------------------------------

def test_quality_measures_hand_example():
    mask = np.array([1, 1, 0, 0, 1, 0, 0, 0], np.uint8)
    truth = np.array([1, 0, 0, 1, 1, 0, 0, 0], np.uint8)
    tp, fp, tn, fn = O.quality_counts(mask, truth)
    assert (tp, fp, tn, fn) == (2, 1, 4, 1)
    q = O.quality_metrics(tp, fp, tn, fn)
    assert q["recall"] == pytest.approx(2 / 3) and q["precision"] == pytest.approx(2 / 3)
    assert q["specificity"] == pytest.approx(4 / 5) and q["fpr"] == pytest.approx(1 / 5)
    assert q["fnr"] == pytest.approx(1 / 3) and q["pwc"] == pytest.approx(100 * 2 / 8)
    assert q["fmeasure"] == pytest.approx(2 / 3)


def test_quality_measures_match_scikit_learn():
    from sklearn.metrics import confusion_matrix, f1_score, precision_score, recall_score
    rng = np.random.default_rng(11)
    truth = rng.random(5000) < 0.1
    mask = truth ^ (rng.random(5000) < 0.05)
    tp, fp, tn, fn = O.quality_counts(mask, truth)
    tn_, fp_, fn_, tp_ = confusion_matrix(truth, mask).ravel()
    assert (tp, fp, tn, fn) == (tp_, fp_, tn_, fn_)
    q = O.quality_metrics(tp, fp, tn, fn)
    assert q["recall"] == pytest.approx(recall_score(truth, mask))
    assert q["precision"] == pytest.approx(precision_score(truth, mask))
    assert q["fmeasure"] == pytest.approx(f1_score(truth, mask))
    assert q["specificity"] + q["fpr"] == pytest.approx(1.0) and q["recall"] + q["fnr"] == pytest.approx(1.0)


def test_roc_sweep_matches_scikit_learn_curve():
    from sklearn.metrics import roc_curve
    rng = np.random.default_rng(12)
    truth = rng.random(3000) < 0.2
    scores = np.abs(rng.standard_normal(3000)) * (1 + 2 * truth)
    fpr, tpr, thr = roc_curve(truth, scores, drop_intermediate=False)
    sel = thr[1:60:7]
    for d, (tp, fp, tn, fn) in zip(sel, O.roc_counts(scores, truth, sel)):
        i = int(np.where(thr == d)[0][0])
        assert fp / (fp + tn) == pytest.approx(fpr[i]) and tp / (tp + fn) == pytest.approx(tpr[i])


def test_pixel_scores_reproduce_the_step3_labels():
    prm = O.Params(9, 7, 3, k=2, mu=1e-3)
    rng = np.random.default_rng(13)
    U = V.random_orthonormal(prm.m, 2, rng)
    y = rng.standard_normal(2)
    x = U @ y + 0.05 * rng.standard_normal(prm.m)
    lab = O.pixel_labels(U, x, y, prm.thr, 3)
    assert np.array_equal(lab, (O.pixel_scores(U, x, y, 3) >= prm.thr).astype(np.uint8))


def test_paper_table_rows_are_consistent_measures():
    """The per-category rows printed in Sec. 5 satisfy Specificity = 1 - FPR
    and FNR = 1 - Recall to the printed precision (tests/golden fixture)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_quality_table.json")
    d = json.load(open(path))
    for row in d["rows"]:
        assert row["specificity"] + row["fpr"] == pytest.approx(1.0, abs=2e-4)
        if row["category"] not in d["inconsistent_fnr"]:
            assert row["recall"] + row["fnr"] == pytest.approx(1.0, abs=2e-3)


# ---------------------------------------------------------------------------
# Step 1 variants: gradient descent with the same step rule
# ---------------------------------------------------------------------------

def test_gradient_descent_variant_on_quadratic_has_orthogonal_gradients():
    """p = 2 makes the cost quadratic, so the majoriser step is the exact
    line minimum: successive steepest-descent gradients are orthogonal, the
    cost decreases every step, and the first step equals CG's."""
    rng = np.random.default_rng(21)
    m, k = 300, 4
    U = V.random_orthonormal(m, k, rng)
    w = np.exp(rng.uniform(-3, 0, m))
    x = rng.standard_normal(m)
    y0 = np.zeros(k)
    ys = []
    for J in range(1, 4):
        y, rec = O.cg_solve(U, x, w, y0, J, 2.0, 1e-3, O.COST_LP, "gd")
        ys.append(y)
        assert all(b <= a + 1e-12 for a, b in zip(rec.f, rec.f[1:]))
    gs = [-(U.T @ (w * O.dphi(x - U @ y, 2.0, 1e-3))) for y in [y0] + ys]
    for a, b in zip(gs, gs[1:]):
        assert abs(a @ b) <= 1e-8 * np.linalg.norm(a) * np.linalg.norm(b)
    y1cg, _ = O.cg_solve(U, x, w, y0, 1, 2.0, 1e-3, O.COST_LP, "cg")
    assert np.allclose(ys[0], y1cg, rtol=0, atol=1e-14)


@pytest.mark.parametrize("seed", [22, 23, 24])
def test_cg_beats_gradient_descent_on_a_quadratic(seed):
    """Sec. 3.3's argument for CG: on a quadratic (p = 2) CG with exact
    steps minimises over the Krylov space that also holds the gradient
    descent iterates, so after the same number of steps its cost is never
    higher (and here lower)."""
    rng = np.random.default_rng(seed)
    m, k = 400, 8
    U = V.random_orthonormal(m, k, rng)
    w = np.exp(rng.uniform(-6, 0, m))
    x = U @ (3 * rng.standard_normal(k)) + 0.1 * rng.standard_normal(m)
    for J in (2, 3, 4):
        _, rc = O.cg_solve(U, x, w, np.zeros(k), J, 2.0, 1e-3, O.COST_LP, "cg")
        _, rg = O.cg_solve(U, x, w, np.zeros(k), J, 2.0, 1e-3, O.COST_LP, "gd")
        assert rc.f[-1] < rg.f[-1]


def test_irls_variant_solves_weighted_least_squares_in_one_step():
    """p = 2: the majoriser is the cost itself, so one IRLS step lands on the
    weighted least-squares solution (numpy lstsq on sqrt(w)-scaled rows)."""
    rng = np.random.default_rng(25)
    m, k = 200, 5
    U = V.random_orthonormal(m, k, rng)
    w = np.exp(rng.uniform(-3, 0, m))
    x = rng.standard_normal(m)
    y, rec = O.cg_solve(U, x, w, rng.standard_normal(k), 1, 2.0, 1e-3, O.COST_LP, "irls")
    sw = np.sqrt(w)
    ref = np.linalg.lstsq(U * sw[:, None], x * sw, rcond=None)[0]
    assert np.allclose(y, ref, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("p", [0.25, 1.0])
def test_irls_variant_is_monotone_and_reaches_a_stationary_point(p):
    rng = np.random.default_rng(26)
    m, k = 300, 4
    U = V.random_orthonormal(m, k, rng)
    w = np.where(rng.random(m) < 0.1, 5e-5, 1.0)
    x = U @ rng.standard_normal(k) + 0.02 * rng.standard_normal(m)
    x[rng.random(m) < 0.1] += 1.0
    y, rec = O.cg_solve(U, x, w, np.zeros(k), 30, p, 1e-3, O.COST_LP, "irls")
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(rec.f, rec.f[1:]))
    g = -(U.T @ (w * O.dphi(x - U @ y, p, 1e-3)))
    g0 = -(U.T @ (w * O.dphi(x, p, 1e-3)))
    assert np.linalg.norm(g) <= 1e-6 * np.linalg.norm(g0)


# --- video ingest: area re-sampling (Sec. 5.1) and mask upsampling (Sec. 5.3) ---

def test_resample_integer_factor_is_the_block_mean():
    """640x480 -> 160x120 (factor 4): each output pixel is the plain mean of
    its 4 x 4 source block."""
    rng = np.random.default_rng(11)
    img = rng.integers(0, 256, size=(48, 64, 3), dtype=np.uint8)
    out = O.resample_area(img, 16, 12, scale=1.0)
    blocks = img.astype(np.float64).reshape(12, 4, 16, 4, 3).mean(axis=(1, 3))
    np.testing.assert_allclose(out, np.moveaxis(blocks, 2, 0).reshape(-1), rtol=0, atol=1e-12)


@pytest.mark.parametrize("src,dst", [((7, 5), (3, 2)), ((5, 7), (4, 3)), ((3, 2), (7, 5)), ((11, 13), (11, 13)),
                                     ((1, 1), (4, 3)), ((9, 4), (1, 1))])
def test_resample_matches_supersampled_block_mean(src, dst):
    """Any sizes: replicating every source pixel dst_h x dst_w times makes each
    destination footprint an exact block of H x W cells, whose plain mean is
    the area average (brute force on tiny inputs)."""
    (W, H), (w, h) = src, dst
    rng = np.random.default_rng(W * 100 + H)
    img = rng.integers(0, 256, size=(H, W, 2), dtype=np.uint8)
    big = np.repeat(np.repeat(img.astype(np.float64), h, axis=0), w, axis=1)
    ref = big.reshape(h, H, w, W, 2).mean(axis=(1, 3))
    out = O.resample_area(img, w, h, scale=1.0)
    np.testing.assert_allclose(out, np.moveaxis(ref, 2, 0).reshape(-1), rtol=0, atol=1e-10)


def test_resample_identity_constant_and_mass():
    rng = np.random.default_rng(5)
    img = rng.integers(0, 256, size=(10, 14, 3), dtype=np.uint8)
    same = O.resample_area(img, 14, 10)
    np.testing.assert_allclose(same, np.moveaxis(img, 2, 0).reshape(-1) / 255.0, rtol=0, atol=1e-15)
    const = O.resample_area(np.full((9, 13, 1), 200, np.uint8), 5, 4)
    np.testing.assert_allclose(const, 200 / 255.0, rtol=1e-15)
    out = O.resample_area(img, 6, 7, scale=1.0).reshape(3, 7, 6)
    # the integral over the image is preserved: mean of each plane unchanged
    np.testing.assert_allclose(out.mean(axis=(1, 2)), img.astype(np.float64).mean(axis=(0, 1)), rtol=1e-12)


def test_mask_upsample_integer_factor_replicates_pixels():
    rng = np.random.default_rng(2)
    m = (rng.random((6, 8)) < 0.3).astype(np.uint8)
    out = O.mask_upsample(m.reshape(-1), 8, 6, 32, 24).reshape(24, 32)
    np.testing.assert_array_equal(out, np.kron(m, np.ones((4, 4), np.uint8)))
    np.testing.assert_array_equal(O.mask_upsample(m.reshape(-1), 8, 6, 8, 6), m.reshape(-1))


def test_mask_upsample_picks_the_pixel_under_each_centre():
    """Non-integer ratio: every output centre falls inside the source pixel
    it copies (checked with exact fractions)."""
    from fractions import Fraction
    rng = np.random.default_rng(4)
    w, h, ow, oh = 7, 5, 16, 9
    m = (rng.random(h * w) < 0.5).astype(np.uint8)
    out = O.mask_upsample(m, w, h, ow, oh).reshape(oh, ow)
    for i in range(oh):
        for j in range(ow):
            cy, cx = Fraction(2 * i + 1, 2) * Fraction(h, oh), Fraction(2 * j + 1, 2) * Fraction(w, ow)
            r, c = int(cy), int(cx)
            assert r <= cy < r + 1 and c <= cx < c + 1
            assert out[i, j] == m[r * w + c]


# --------------------------------------------------------------------------
# small helpers, each against its definition written out entry by entry
# --------------------------------------------------------------------------

def test_pixel_weights_planar_layout_by_loops():
    """eq. (pixelweighting): entry c*P + p of the weight vector is 1 when
    pixel p was background in the previous frame and omega otherwise, for
    every colour plane c."""
    rng = _rng(31)
    P, C, omega = 37, 3, 0.125
    lab = (rng.random(P) < 0.3).astype(np.uint8)
    w = O.pixel_weights(lab, omega, C)
    assert w.shape == (C * P,)
    for c in range(C):
        for p in range(P):
            assert w[c * P + p] == (omega if lab[p] else 1.0)


def test_cho_solve_lower_solves_the_normal_equations():
    rng = _rng(32)
    B = rng.standard_normal((6, 6))
    A = B @ B.T + 6 * np.eye(6)
    b = rng.standard_normal(6)
    z = O.cho_solve_lower(np.linalg.cholesky(A), b)
    np.testing.assert_allclose(A @ z, b, rtol=0, atol=1e-12)


def test_band_pixels_by_loops():
    """A pixel is in the band when its largest channel residual lies within
    the guard of the threshold (brute force over pixels and channels)."""
    rng = _rng(33)
    P, C, k = 50, 3, 2
    U = V.random_orthonormal(C * P, k, rng)
    y = rng.standard_normal(k)
    x = U @ y + 0.1 * rng.standard_normal(C * P)
    thr, guard = 0.1, 0.03
    got = O.band_pixels(U, x, y, thr, C, guard)
    r = x - U @ y
    for p in range(P):
        rmax = max(abs(r[c * P + p]) for c in range(C))
        assert bool(got[p]) == (abs(rmax - thr) <= guard)
    assert 0 < got.sum() < P


# --------------------------------------------------------------------------
# diagnostics: orthonormality error and principal angles (Sec. 2.1,
# eq. stiefeldef); they are the checkers of the trajectory pins above
# --------------------------------------------------------------------------

def _plane_pair(m, thetas, seed):
    """Orthonormal A, B (m x len(thetas)) whose principal angles are exactly
    thetas: A_i = cos(t_i) e_i + sin(t_i) f_i, B_i = e_i, with e, f the
    columns of one orthonormal basis."""
    a = len(thetas)
    E, _ = np.linalg.qr(_rng(seed).standard_normal((m, 2 * a)))
    B = E[:, :a]
    A = np.cos(thetas)[None, :] * B + np.sin(thetas)[None, :] * E[:, a:]
    return A, B


def test_principal_angles_known_rotation_including_tiny():
    """Planes rotated by known angles, down to 1e-7 rad (where an arccos
    form loses all digits), come back as those angles."""
    thetas = np.array([1e-7, 3e-4, 0.25, 1.1, np.pi / 2])
    A, B = _plane_pair(40, thetas, 31)
    got = np.sort(O.principal_angles(A, B))
    np.testing.assert_allclose(got, np.sort(thetas), rtol=1e-8, atol=1e-15)
    assert got[0] > 0.5e-7   # not lost to cancellation


def test_principal_angles_against_scipy_subspace_angles():
    """Random subspaces of unequal dimension: the same angles as
    scipy.linalg.subspace_angles."""
    rng = _rng(32)
    A, _ = np.linalg.qr(rng.standard_normal((30, 3)))
    B, _ = np.linalg.qr(rng.standard_normal((30, 5)))
    got = np.sort(O.principal_angles(A, B))
    ref = np.sort(scipy.linalg.subspace_angles(A, B))
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-13)


def test_principal_angles_contained_and_orthogonal():
    """A vector inside span(B) makes angle 0; one orthogonal to it pi/2;
    a basis change of the same span does not move the angles."""
    rng = _rng(33)
    B, _ = np.linalg.qr(rng.standard_normal((25, 4)))
    inside = B @ rng.standard_normal(4)
    inside /= np.linalg.norm(inside)
    assert O.principal_angles(inside[:, None], B)[0] < 1e-14
    out = rng.standard_normal(25)
    out -= B @ (B.T @ out)
    out /= np.linalg.norm(out)
    assert abs(O.principal_angles(out[:, None], B)[0] - np.pi / 2) < 1e-7
    Qr, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    assert O.principal_angles(B @ Qr, B).max() < 1e-7


def test_orthonormality_error_by_loops_and_planted_scaling():
    """||U^T U - I||_F against an explicit double loop over column pairs,
    and a planted column scaling diag(1 + eps) of an orthonormal U, whose
    error is sqrt(sum((1 + eps_i)^2 - 1)^2) in closed form."""
    rng = _rng(34)
    U = rng.standard_normal((20, 4)) * 0.5
    tot = 0.0
    for i in range(4):
        for j in range(4):
            dot = sum(U[e, i] * U[e, j] for e in range(20))
            tot += (dot - (1.0 if i == j else 0.0)) ** 2
    assert abs(O.orthonormality_error(U) - math.sqrt(tot)) < 1e-13 * max(1.0, math.sqrt(tot))
    Q, _ = np.linalg.qr(rng.standard_normal((50, 5)))
    eps = np.array([1e-3, -2e-4, 0.0, 5e-6, 0.3])
    want = math.sqrt(float(np.sum(((1 + eps) ** 2 - 1) ** 2)))
    assert abs(O.orthonormality_error(Q * (1 + eps)[None, :]) - want) < 1e-12
    assert O.orthonormality_error(Q) < 1e-14
    # a planted off-diagonal: rotate column 1 towards column 0 without renormalising
    V_ = Q.copy()
    V_[:, 1] = Q[:, 1] + 1e-4 * Q[:, 0]
    want = math.sqrt(2 * 1e-4 ** 2 + (1e-4 ** 2) ** 2)
    assert abs(O.orthonormality_error(V_) - want) < 1e-12


# ---------------------------------------------------------------------------
# Initialization of U (Sec. 3.4): Q of the reduced QR of a random matrix,
# drawn from Philox4x32-10 + Box-Muller
# ---------------------------------------------------------------------------

def test_philox_known_answers():
    import json
    kat = json.load(open(os.path.join(GOLD, "philox4x32_10_kat.json")))
    for v in kat["vectors"]:
        ctr = np.array([int(w, 16) for w in v["ctr"]], dtype=np.uint64)
        key = [int(w, 16) for w in v["key"]]
        out = O.philox4x32_10(ctr, key)
        assert [int(w) for w in out] == [int(w, 16) for w in v["out"]]


def test_philox_is_counter_based():
    """Vectorised calls equal one call per counter; a changed key or counter
    word changes every output word."""
    ctr = np.array([[q, 7, 3, 0] for q in range(50)], dtype=np.uint64)
    many = O.philox4x32_10(ctr, (11, 12))
    for q in range(50):
        assert np.array_equal(many[q], O.philox4x32_10(ctr[q], (11, 12)))
    a = O.philox4x32_10(np.array([1, 2, 3, 4]), (5, 6))
    for alt in (O.philox4x32_10(np.array([1, 2, 3, 5]), (5, 6)), O.philox4x32_10(np.array([1, 2, 3, 4]), (5, 7))):
        assert np.all(a != alt)


def test_gaussian_matrix_is_standard_normal():
    """Moments and a Kolmogorov-Smirnov test against N(0, 1) on 200 000
    draws; the cosine and sine variates of a pair are uncorrelated; the
    column-major layout is the linear draw order."""
    from scipy import stats
    A = O.gaussian_matrix(40000, 5, seed=2024)
    g = A.T.ravel()                     # draw order e = j m + i
    assert abs(g.mean()) < 0.01 and abs(g.var() - 1.0) < 0.01
    assert abs(np.mean(g ** 4) - 3.0) < 0.05
    assert stats.kstest(g, "norm").pvalue > 1e-3
    assert abs(np.corrcoef(g[0::2], g[1::2])[0, 1]) < 0.01
    B = O.gaussian_matrix(40000, 5, seed=2024, stream=1)
    assert abs(np.corrcoef(A.ravel(), B.ravel())[0, 1]) < 0.01
    # a smaller matrix is a prefix of the same draw order
    assert np.array_equal(O.gaussian_matrix(10, 3, seed=9).T.ravel(), O.gaussian_matrix(15, 2, seed=9).T.ravel()[:30])


def test_initial_subspace_is_the_reduced_qr_factor():
    """U0 has orthonormal columns, spans the random matrix's column space,
    and R = U0^T A is upper triangular with a positive diagonal (the unique
    reduced QR); odd m k (the last draw pair half used) included."""
    for (m, k, seed) in ((4801, 5, 1), (300, 16, 2), (7, 7, 3), (1000, 1, 4)):
        A = O.gaussian_matrix(m, k, seed)
        U = O.initial_subspace(m, k, seed)
        assert O.orthonormality_error(U) < 1e-13
        R = U.T @ A
        assert np.all(np.diag(R) > 0)
        assert np.max(np.abs(np.tril(R, -1))) < 1e-12 * np.max(np.abs(R))
        assert np.max(np.abs(U @ R - A)) < 1e-12 * np.max(np.abs(A))
    assert not np.allclose(O.initial_subspace(100, 3, 1), O.initial_subspace(100, 3, 1, stream=1))
