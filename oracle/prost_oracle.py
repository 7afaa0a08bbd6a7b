"""FP64 CPU oracle for pROST's per-frame alternating minimisation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
executes this module; only the tests, the smoke check and the CPU-baseline
leg of the benchmark do.  It shares no code with the HIP library.

Paper: Seidel, Hage, Kleinsteuber, "pROST: A Smoothed lp-norm Robust Online
Subspace Tracking Method for Realtime Background Subtraction in Video"
(arXiv:1302.2073).  Every function below cites the passage it follows.

Conventions
-----------
* A frame x is a vector of m = C*P entries stored plane by plane
  (all P pixels of channel 0, then channel 1, ...), each plane row-major
  over an H x W image, as in Sec. 3.4 "Color images" (x = [x_R; x_G; x_B]).
  Pixel index p = row*W + col; entry index e = c*P + p.
* U is m x k with orthonormal columns (Sec. 2.1, eq. stiefeldef), y in R^k.
* All arithmetic is float64, sums are numpy's (pairwise) sums.  There is no
  blocking, fusion or reordering beyond the definitions.

Readings of points the paper leaves open are marked READING and listed in
the design notes of the repository.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

COST_LP = "lp"    # eq. (smoothlpnorm): (r^2 + mu)^(p/2)
COST_LOG = "log"  # log(1 + r^2/mu), the p -> 0 limit of the lp form (shifted, rescaled)


# ---------------------------------------------------------------------------
# Cost functor, Sec. 3.1, eqs. (smoothlpnorm), (weightedLPnorm)
# ---------------------------------------------------------------------------

def phi(r, p, mu, form=COST_LP):
    """Per-entry smoothed cost.  lp form: eq. (smoothlpnorm) summand
    (r^2+mu)^(p/2).  log form: log(1 + r^2/mu)."""
    r = np.asarray(r, dtype=np.float64)
    if form == COST_LP:
        return (r * r + mu) ** (p / 2.0)
    if form == COST_LOG:
        return np.log1p(r * r / mu)
    raise ValueError(form)


def dphi(r, p, mu, form=COST_LP):
    """d phi / d r.  lp form: p r (r^2+mu)^(p/2-1), the factor appearing in the
    derivative of Sec. 3.3 (Step 2).  log form: 2r/(mu+r^2)."""
    r = np.asarray(r, dtype=np.float64)
    if form == COST_LP:
        return p * r * (r * r + mu) ** (p / 2.0 - 1.0)
    if form == COST_LOG:
        return 2.0 * r / (mu + r * r)
    raise ValueError(form)


def curv(r, p, mu, form=COST_LP):
    """c(r) = phi'(r)/r, the weight of the quadratic majoriser of phi at r
    (phi is a concave function of r^2 for p <= 2, Sec. 3.1)."""
    r = np.asarray(r, dtype=np.float64)
    if form == COST_LP:
        return p * (r * r + mu) ** (p / 2.0 - 1.0)
    if form == COST_LOG:
        return 2.0 / (mu + r * r)
    raise ValueError(form)


def dphi_dmu(r, p, mu, form=COST_LP):
    """d phi / d mu, needed by the differentiable cost."""
    r = np.asarray(r, dtype=np.float64)
    if form == COST_LP:
        return (p / 2.0) * (r * r + mu) ** (p / 2.0 - 1.0)
    if form == COST_LOG:
        return -(r * r) / (mu * (mu + r * r))
    raise ValueError(form)


def delta_from_mu(mu, p, form=COST_LP):
    """Threshold delta at which the second derivative of the cost in r
    vanishes, eqs. (opt_mu), (opt_mu2): mu = delta^2 (1-p) for the lp form,
    so delta = sqrt(mu/(1-p)).  For the log form the inflection is at
    sqrt(mu) (the same condition applied to log(1+r^2/mu))."""
    if form == COST_LP:
        return math.sqrt(mu / (1.0 - p))
    return math.sqrt(mu)


def mu_from_delta(delta, p):
    """eq. (opt_mu2): mu = delta^2 (1 - p)."""
    return delta * delta * (1.0 - p)


# ---------------------------------------------------------------------------
# Parameters and state
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Params:
    """Parameter set of Sec. 5.1 (k, omega, t_init, t_min, delta, p, mu and the
    number of CG steps).  Defaults are the benchmark values printed there,
    except mu/delta which callers set per workload."""
    width: int
    height: int
    channels: int = 1
    k: int = 15
    cg_iters: int = 5            # "a maximum of five CG steps" (Sec. 5.1)
    cost: str = COST_LP
    p: float = 0.25
    mu: float = 1e-3
    delta: Optional[float] = None  # None -> delta_from_mu (eq. opt_mu2)
    omega: float = 5e-5
    t_init: float = 5e-3
    t_min: float = 1e-4
    i_init: int = 100
    labels_after_update: bool = True   # READING: step 3 uses U^(i+1)
    weights_from_filtered: bool = False  # READING: raw labels feed the weights
    preprocess: bool = False     # Sec. 3.4 pre-processing (mean subtraction, scaling)
    ysolve: str = "cg"           # Step 1 solver: "cg" (PR+), "gd" (gradient descent), "irls" (-H^-1 g)

    @property
    def P(self):
        return self.width * self.height

    @property
    def m(self):
        return self.channels * self.P

    @property
    def thr(self):
        return self.delta if self.delta is not None else delta_from_mu(self.mu, self.p, self.cost)


@dataclasses.dataclass
class Preproc:
    """Statistics of the pre-processing of Sec. 3.4 (Pre- and
    post-processing) over the frames of the initialization phase seen so
    far: per-entry sums of x and x^2 (float64) and the frame count."""
    s1: np.ndarray       # m, sum of x
    s2: np.ndarray       # m, sum of x^2
    count: int = 0

    def copy(self):
        return Preproc(self.s1.copy(), self.s2.copy(), self.count)

    @property
    def mean(self):
        return self.s1 / self.count if self.count else np.zeros_like(self.s1)

    @property
    def m2(self):
        """Per-entry sum of squared deviations from the per-entry mean."""
        if not self.count:
            return np.zeros_like(self.s1)
        return self.s2 - self.s1 * self.s1 / self.count


def preproc_init(m):
    return Preproc(np.zeros(m), np.zeros(m), 0)


def preproc_scale(pp: Preproc):
    """Sample standard deviation over all entries of the initialization
    frames seen so far, of the mean-subtracted values (READING: pooled
    within-entry variance, sum of squared deviations / (m (N - 1)));
    1 while fewer than two frames are in (or the variance is 0)."""
    if pp.count < 2:
        return 1.0
    var = float(pp.m2.sum()) / (pp.s1.size * (pp.count - 1))
    return math.sqrt(var) if var > 0.0 else 1.0


def preprocess(pp: Preproc, x, n, i_init):
    """Sec. 3.4 pre-processing of frame n: while n < i_init (the
    initialization phase of the step-size rule) the frame joins the running
    average; the frame minus the running average (this frame included) is
    divided by the standard deviation of the initialization frames before
    this one (READING: the pooled deviation is a reduction over the whole
    frame, so the current frame's contribution counts from the next frame
    on).  After the initialization phase both are frozen.  Returns
    (x_tilde, new statistics)."""
    x = np.asarray(x, dtype=np.float64)
    s = preproc_scale(pp)
    if n < i_init:
        pp = Preproc(pp.s1 + x, pp.s2 + x * x, pp.count + 1)
    return (x - pp.mean) / s, pp


@dataclasses.dataclass
class State:
    U: np.ndarray        # m x k
    y: np.ndarray        # k
    labels: np.ndarray   # P, uint8 raw labels of the previous frame
    mask: np.ndarray     # P, uint8 median-filtered mask of the previous frame
    n: int = 0           # number of frames processed
    pre: Optional[Preproc] = None   # pre-processing statistics (when enabled)

    def copy(self):
        return State(self.U.copy(), self.y.copy(), self.labels.copy(), self.mask.copy(), self.n,
                     None if self.pre is None else self.pre.copy())


def initial_state(U0, P):
    """Start of the online scheme, Sec. 3.4 (Initialization): U0 given
    (a reduced QR of a random matrix, drawn by the caller); y = 0; no pixel
    labelled foreground yet."""
    U0 = np.array(U0, dtype=np.float64)
    k = U0.shape[1]
    return State(U0, np.zeros(k), np.zeros(P, np.uint8), np.zeros(P, np.uint8), 0)


# ---------------------------------------------------------------------------
# Weighted cost and its pieces, eqs. (weightedLPnorm), (spcacost)
# ---------------------------------------------------------------------------

def pixel_weights(labels, omega, channels):
    """eq. (pixelweighting): weight 1 where the previous frame's label is
    background, omega where it is foreground.  READING: one weight per pixel,
    shared by all colour entries of that pixel."""
    wp = np.where(np.asarray(labels) == 0, 1.0, float(omega))
    return np.tile(wp, channels)


def cost(U, x, y, w, p, mu, form=COST_LP):
    """h_{mu,w}(x - U y), eq. (spcacost)."""
    r = x - U @ y
    return float(np.sum(w * phi(r, p, mu, form)))


def grad_y(U, x, y, w, p, mu, form=COST_LP):
    """Gradient of eq. (spcacost) in y: -U^T (w * phi'(r)), r = x - U y."""
    r = x - U @ y
    return -(U.T @ (w * dphi(r, p, mu, form)))


def curvature(U, x, y, w, p, mu, form=COST_LP):
    """H = U^T diag(w * c(r)) U: curvature of the quadratic majoriser of
    eq. (spcacost) at y (c = phi'/r)."""
    r = x - U @ y
    cw = w * curv(r, p, mu, form)
    return U.T @ (U * cw[:, None])


# ---------------------------------------------------------------------------
# Step 1: y-solve, eq. (onlinestep1), CG of Sec. 3.3
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class CGRecord:
    f: list            # cost at y_0 .. y_J (f[-1] at the returned y)
    alpha: list
    beta: list
    restarts: int
    iters: int


def cho_solve_lower(L, b):
    """Solve (L L^T) z = b by two triangular solves (library routines)."""
    import scipy.linalg
    return scipy.linalg.solve_triangular(L.T, scipy.linalg.solve_triangular(L, b, lower=True), lower=False)


def cg_solve(U, x, w, y0, J, p, mu, form=COST_LP, method="cg"):
    """Minimise h_{mu,w}(x - U y) over y from the warm start y0 with at most J
    nonlinear conjugate-gradient steps (Sec. 3.3 Step 1; J = 5, Sec. 5.1).
    method = "gd": plain gradient descent with the same step rule (the
    simpler alternative Sec. 3.3 compares CG with).  method = "irls": the
    full majoriser step, y += -H^{-1} g (iteratively reweighted least
    squares / Newton on the majoriser); stops when H is not positive
    definite.

    READING (the paper names CG but not its variant or line search):
    Polak-Ribiere-plus direction, restart along -g when the direction is not
    a descent direction, and the step alpha = -g.d / (d.H d) that minimises
    the quadratic majoriser f + a g.d + a^2/2 d.H d of the cost along d
    (H from `curvature`), so the cost never increases.  A fixed number of
    steps; stop early only at an exactly zero gradient or zero curvature."""
    y = np.array(y0, dtype=np.float64)
    rec = CGRecord([], [], [], 0, 0)
    g_prev = d_prev = None
    for j in range(J):
        r = x - U @ y
        rec.f.append(float(np.sum(w * phi(r, p, mu, form))))
        g = -(U.T @ (w * dphi(r, p, mu, form)))
        if not np.any(g):
            break
        if method == "irls":
            H = U.T @ (U * (w * curv(r, p, mu, form))[:, None])
            try:
                L = np.linalg.cholesky(H)
            except np.linalg.LinAlgError:
                break
            y = y - cho_solve_lower(L, g)
            rec.alpha.append(1.0)
            rec.beta.append(0.0)
            rec.iters += 1
            continue
        if j == 0 or method == "gd":
            d = -g
            beta = 0.0
        else:
            beta = max(0.0, float(g @ (g - g_prev)) / float(g_prev @ g_prev))
            d = -g + beta * d_prev
            if float(g @ d) >= 0.0:
                d = -g
                rec.restarts += 1
        H = U.T @ (U * (w * curv(r, p, mu, form))[:, None])
        dHd = float(d @ H @ d)
        if not dHd > 0.0:
            break
        alpha = -float(g @ d) / dHd
        y = y + alpha * d
        rec.alpha.append(alpha)
        rec.beta.append(beta)
        rec.iters += 1
        g_prev, d_prev = g, d
    rec.f.append(cost(U, x, y, w, p, mu, form))
    return y, rec


# ---------------------------------------------------------------------------
# Step 2: one geodesic step on the Grassmannian, Sec. 3.2, 3.3
# ---------------------------------------------------------------------------

def project_tangent(U, H):
    """eq. (gproject): pi(H) = (I - U U^T) H."""
    return H - U @ (U.T @ H)


def step_size(n, t_init, t_min, i_init):
    """Step-size rule of Sec. 3.4: t = max(exp(-tau i) t_init, t_min) with
    tau = -log(t_min/t_init) / i_init.  READING: i is the 0-based frame
    index."""
    tau = -math.log(t_min / t_init) / i_init
    return max(math.exp(-tau * n) * t_init, t_min)


def eta_vector(U, x, y, w, p, mu, form=COST_LP):
    """eta_i = -p w_i r_i (r_i^2+mu)^(p/2-1) = -w_i phi'(r_i), r = x - U y
    (Sec. 3.3 Step 2); the Euclidean gradient in U is eta y^T."""
    r = x - U @ y
    return -w * dphi(r, p, mu, form)


def rank_one_svd(U, eta, y):
    """Closed-form SVD of the projected gradient G_U = pi(eta) y^T, eq. (svd):
    s = pi(eta)/||pi(eta)||, sigma = ||pi(eta)|| ||y||, v = y/||y||.
    The projection is applied twice so that s is orthogonal to span(U) to
    working precision.  Returns (s, sigma, v, zeta, nu) with zeta =
    ||pi(eta)|| and nu = ||y||; s or v is None when zeta or nu is 0."""
    z = project_tangent(U, eta)
    z = project_tangent(U, z)
    zeta = float(np.linalg.norm(z))
    nu = float(np.linalg.norm(y))
    s = z / zeta if zeta > 0 else None
    v = y / nu if nu > 0 else None
    return s, zeta * nu, v, zeta, nu


def geodesic_rank_one(U, s, v, theta):
    """eq. (geodesic) for the descent direction B = -G_U = sigma (-s) v^T.
    The thin SVD of B completes v to an orthonormal V in O(k) (all other
    singular values are zero), which leaves
        U(t) = U + (cos(theta) - 1) (U v) v^T - sin(theta) s v^T,
    theta = sigma t.  READING: the "compact SVD" of the paper is taken as
    this thin SVD; a literal rank-one compact SVD would collapse U(t)."""
    Uv = U @ v
    return U + (math.cos(theta) - 1.0) * np.outer(Uv, v) - math.sin(theta) * np.outer(s, v)


# ---------------------------------------------------------------------------
# Step 3: segmentation and weights, Sec. 3.3 Step 3, Sec. 3.4
# ---------------------------------------------------------------------------

def pixel_labels(U, x, y, thr, channels):
    """Label a pixel foreground when the largest residual over its colour
    channels reaches the threshold, Sec. 3.4 (Color images);
    eq. (pixelweighting) for one channel.  READING: ties (== thr) are
    foreground, as in the colour rule."""
    r = np.abs(x - U @ y)
    P = r.size // channels
    rmax = r.reshape(channels, P).max(axis=0)
    return (rmax >= thr).astype(np.uint8)


def median3x3(labels, height, width):
    """3x3 median filter of the binary mask (Sec. 3.4, Pre- and
    post-processing).  On binary values the median of the nine neighbours is
    1 exactly when at least five of them are 1.  READING: image borders
    replicate the edge pixel."""
    L = np.asarray(labels, dtype=np.int64).reshape(height, width)
    pad = np.pad(L, 1, mode="edge")
    acc = np.zeros_like(L)
    for di in range(3):
        for dj in range(3):
            acc += pad[di:di + height, dj:dj + width]
    return (acc >= 5).astype(np.uint8).reshape(-1)


# ---------------------------------------------------------------------------
# One frame of the online alternating minimisation, Sec. 3.3
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class FrameInfo:
    cg: CGRecord
    t: float
    sigma: float
    theta: float
    zeta: float
    nu: float
    updated: bool
    x: Optional[np.ndarray] = None   # the frame the steps ran on (pre-processed if enabled)


def track_frame(state: State, x, prm: Params):
    """Process frame x (length m): Step 1 refines y from the previous y,
    Step 2 takes one geodesic step on U, Step 3 labels the pixels (Sec. 3.3),
    followed by the 3x3 median (Sec. 3.4).  Returns (new_state, info)."""
    x = np.asarray(x, dtype=np.float64)
    pre = state.pre
    if prm.preprocess:
        x, pre = preprocess(pre if pre is not None else preproc_init(x.size), x, state.n, prm.i_init)
    U = state.U
    src = state.mask if prm.weights_from_filtered else state.labels
    w = pixel_weights(src, prm.omega, prm.channels)
    # Step 1
    y, rec = cg_solve(U, x, w, state.y, prm.cg_iters, prm.p, prm.mu, prm.cost, prm.ysolve)
    # Step 2
    eta = eta_vector(U, x, y, w, prm.p, prm.mu, prm.cost)
    s, sigma, v, zeta, nu = rank_one_svd(U, eta, y)
    t = step_size(state.n, prm.t_init, prm.t_min, prm.i_init)
    theta = sigma * t
    updated = s is not None and v is not None   # READING: no step when G_U = 0
    U_new = geodesic_rank_one(U, s, v, theta) if updated else U.copy()
    # Step 3
    U_lab = U_new if prm.labels_after_update else U
    labels = pixel_labels(U_lab, x, y, prm.thr, prm.channels)
    mask = median3x3(labels, prm.height, prm.width)
    new = State(U_new, y, labels, mask, state.n + 1, pre)
    return new, FrameInfo(rec, t, sigma, theta, zeta, nu, updated, x)


# ---------------------------------------------------------------------------
# Video ingest: every sequence is re-sampled to one small resolution before
# tracking (Sec. 5.1, 160 x 120), and the mask is brought back to the
# source resolution for evaluation (Sec. 5.3, "Subspace dimension")
# ---------------------------------------------------------------------------

def _box_weights(n_src, n_dst):
    """W[i, s] = length of the overlap of source cell [s, s+1) with the
    footprint [i*n_src/n_dst, (i+1)*n_src/n_dst) of destination cell i,
    divided by the footprint length (rows of W sum to 1)."""
    step = n_src / n_dst
    W = np.zeros((n_dst, n_src))
    for i in range(n_dst):
        a, b = i * step, (i + 1) * step
        for s in range(int(math.floor(a)), min(n_src, int(math.ceil(b)))):
            W[i, s] = max(0.0, min(b, s + 1.0) - max(a, float(s)))
    return W / step


def resample_area(img, dst_w, dst_h, scale=1.0 / 255.0):
    """READING: the paper re-samples every video to 160 x 120 without naming
    the filter; taken as area averaging (each destination pixel is the mean
    of the source image, piecewise constant over its pixels, over the
    destination pixel's footprint), the filter that neither aliases nor
    drops pixels when shrinking.  img: H x W x C (interleaved, e.g. uint8
    RGB as a decoder delivers it).  Returns the tracker's frame layout:
    C planes of dst_h x dst_w, times `scale`, flattened (entry c*P + p)."""
    a = np.asarray(img, dtype=np.float64)
    if a.ndim == 2:
        a = a[:, :, None]
    H, W, C = a.shape
    Wy, Wx = _box_weights(H, dst_h), _box_weights(W, dst_w)
    planes = [Wy @ a[:, :, c] @ Wx.T for c in range(C)]
    return (scale * np.stack(planes)).reshape(-1)


def mask_upsample(mask, width, height, out_w, out_h):
    """READING: the mask is brought to a larger (or any) resolution by
    nearest neighbour: output pixel (i, j) takes the label of the source
    pixel that contains its centre ((i + 1/2) h / out_h, (j + 1/2) w / out_w),
    in exact integer arithmetic."""
    m = np.asarray(mask, dtype=np.uint8).reshape(height, width)
    rows = [((2 * i + 1) * height) // (2 * out_h) for i in range(out_h)]
    cols = [((2 * j + 1) * width) // (2 * out_w) for j in range(out_w)]
    return m[np.ix_(rows, cols)].reshape(-1)


# ---------------------------------------------------------------------------
# Segmentation quality against a ground-truth mask (the measures of Sec. 5,
# changedetection.net: Recall, Specificity, FPR, FNR, PWC, Precision,
# F-measure) and the threshold sweep behind its ROC curves
# ---------------------------------------------------------------------------

def quality_counts(mask, truth):
    """(TP, FP, TN, FN) of a binary mask against the ground truth."""
    m = np.asarray(mask).astype(bool).ravel()
    t = np.asarray(truth).astype(bool).ravel()
    return (int(np.sum(m & t)), int(np.sum(m & ~t)), int(np.sum(~m & ~t)), int(np.sum(~m & t)))


def quality_metrics(tp, fp, tn, fn):
    """The seven measures from the four counts (nan where undefined)."""
    def div(a, b):
        return a / b if b else float("nan")
    recall = div(tp, tp + fn)
    precision = div(tp, tp + fp)
    f = div(2.0 * precision * recall, precision + recall) if tp else (0.0 if (fp or fn) else float("nan"))
    return dict(recall=recall, specificity=div(tn, tn + fp), fpr=div(fp, fp + tn), fnr=div(fn, tp + fn),
                pwc=div(100.0 * (fn + fp), tp + fn + fp + tn), precision=precision, fmeasure=f)


def pixel_scores(U, x, y, channels):
    """Per-pixel score max_c |x_c - u_c^T y| whose comparison with delta is
    the Step 3 label (Sec. 3.4 color rule)."""
    r = np.abs(np.asarray(x, np.float64) - U @ y)
    return r.reshape(channels, -1).max(axis=0)


def roc_counts(scores, truth, thresholds):
    """Counts (TP, FP, TN, FN) for labels [score >= delta] at each threshold:
    the delta sweep of Sec. 5 (points FPR, Recall of the ROC curve)."""
    return [quality_counts(np.asarray(scores) >= d, truth) for d in thresholds]


def band_pixels(U, x, y, thr, channels, guard):
    """Pixels whose largest channel residual lies within `guard` of the
    threshold: the only pixels whose label may legitimately differ between
    two correct implementations that round differently."""
    r = np.abs(x - U @ y)
    P = r.size // channels
    rmax = r.reshape(channels, P).max(axis=0)
    return np.abs(rmax - thr) <= guard


# ---------------------------------------------------------------------------
# Precision form: nearest orthonormal basis (re-orthonormalisation)
# ---------------------------------------------------------------------------

def lowdin(U):
    """Nearest matrix with orthonormal columns (polar factor) U G^{-1/2},
    G = U^T U, and the factor G^{1/2} that keeps U y unchanged to first order
    (y <- G^{1/2} y).  Keeps [U] on the Grassmannian (Sec. 3.2: only the
    span matters) with the smallest change of basis."""
    G = U.T @ U
    lam, Q = np.linalg.eigh(G)
    Gm = (Q / np.sqrt(lam)) @ Q.T
    Gp = (Q * np.sqrt(lam)) @ Q.T
    return U @ Gm, Gp


# ---------------------------------------------------------------------------
# Differentiable cost h_mu,w(x - U y) for a batch of frames
# ---------------------------------------------------------------------------

def lpcost_forward(U, Y, X, w, p, mu, form=COST_LP):
    """f_b = sum_e w_e phi(X[e,b] - u_e^T Y[:,b]), eqs. (weightedLPnorm),
    (spcacost), for each column b.  U: m x k, Y: k x B, X: m x B, w: m."""
    R = X - U @ Y
    return (w[:, None] * phi(R, p, mu, form)).sum(axis=0)


def lpcost_backward(U, Y, X, w, p, mu, gout, form=COST_LP):
    """Adjoint of lpcost_forward for an upstream gradient gout (length B).
    dX = gout * w phi'(R); dY = -U^T (w phi'(R)) gout; dU = -(w phi'(R) gout) Y^T
    (for one frame with gout = 1, -dU is the eta y^T of Sec. 3.3);
    dmu = sum_b gout_b sum_e w_e dphi/dmu."""
    R = X - U @ Y
    D = w[:, None] * dphi(R, p, mu, form)
    Dg = D * gout[None, :]
    dX = Dg
    dY = -(U.T @ Dg)
    dU = -(Dg @ Y.T)
    dmu = float(np.sum((w[:, None] * dphi_dmu(R, p, mu, form)) * gout[None, :]))
    return dX, dU, dY, dmu


# ---------------------------------------------------------------------------
# Diagnostics
# ---------------------------------------------------------------------------

def orthonormality_error(U):
    """||U^T U - I||_F (Sec. 2.1, eq. stiefeldef)."""
    k = U.shape[1]
    return float(np.linalg.norm(U.T @ U - np.eye(k)))


def principal_angles(A, B):
    """Principal angles between span(A) (orthonormal, m x a) and span(B)
    (orthonormal, m x b, b >= a), from the singular values of the part of A
    outside span(B) (arcsin form, accurate for small angles)."""
    R = A - B @ (B.T @ A)
    sv = np.linalg.svd(R, compute_uv=False)
    return np.arcsin(np.clip(sv, 0.0, 1.0))


# ---------------------------------------------------------------------------
# Initialization of U, Sec. 3.4 ("Initialization"): the orthonormal factor of
# the reduced QR decomposition of a random m x k matrix.  The random matrix is
# drawn from a counter-based generator so that the HIP library, which draws
# it on the device, can be compared entry by entry: each side implements the
# generator from its published definition and nothing else is shared.
# ---------------------------------------------------------------------------

_PHILOX_M0, _PHILOX_M1 = 0xD2511F53, 0xCD9E8D57   # round multipliers
_PHILOX_W0, _PHILOX_W1 = 0x9E3779B9, 0xBB67AE85   # key schedule (Weyl) increments
_MASK32 = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel random
    numbers: as easy as 1, 2, 3", SC'11).  ctr: (..., 4) uint32 counters,
    key: (2,) uint32.  Each round multiplies words 0 and 2 by the two
    constants (64-bit products), and the new words are
    (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0));
    the key is bumped by the Weyl increments between rounds."""
    c = np.array(ctr, dtype=np.uint64) & _MASK32
    k0, k1 = int(key[0]) & _MASK32, int(key[1]) & _MASK32
    c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _PHILOX_W0) & _MASK32
            k1 = (k1 + _PHILOX_W1) & _MASK32
        p0 = c0 * np.uint64(_PHILOX_M0)          # exact: both factors < 2^32
        p1 = c2 * np.uint64(_PHILOX_M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(_MASK32)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(_MASK32)
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0)
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def gaussian_matrix(m, k, seed, stream=0):
    """The m x k standard normal matrix behind U0.  Entry (i, j) has linear
    index e = j m + i (column-major).  Pair q = e // 2 is one Philox4x32-10
    call with counter (q mod 2^32, q div 2^32, stream, 0) and key
    (seed mod 2^32, seed div 2^32); its words give two uniforms in (0, 1),
    u = ((w0 2^32 + w1) div 2^11 + 1/2) 2^-53 and likewise from (w2, w3), and
    Box-Muller turns them into sqrt(-2 ln u_a) cos(2 pi u_b) (even e) and
    sqrt(-2 ln u_a) sin(2 pi u_b) (odd e)."""
    n = m * k
    q = np.arange((n + 1) // 2, dtype=np.uint64)
    ctr = np.stack([q & np.uint64(_MASK32), q >> np.uint64(32),
                    np.full_like(q, stream & _MASK32), np.zeros_like(q)], axis=-1)
    w = philox4x32_10(ctr, (seed & _MASK32, (seed >> 32) & _MASK32)).astype(np.uint64)
    za = ((w[:, 0] << np.uint64(32)) | w[:, 1]) >> np.uint64(11)
    zb = ((w[:, 2] << np.uint64(32)) | w[:, 3]) >> np.uint64(11)
    ua = (za.astype(np.float64) + 0.5) * 2.0 ** -53
    ub = (zb.astype(np.float64) + 0.5) * 2.0 ** -53
    rad = np.sqrt(-2.0 * np.log(ua))
    g = np.empty(2 * len(q))
    g[0::2] = rad * np.cos(2.0 * np.pi * ub)
    g[1::2] = rad * np.sin(2.0 * np.pi * ub)
    return g[:n].reshape(k, m).T.copy()


def initial_subspace(m, k, seed, stream=0):
    """U0 of Sec. 3.4: the Q factor of the reduced QR decomposition of the
    random matrix, signs fixed so that diag(R) > 0 (the factorisation is then
    unique)."""
    A = gaussian_matrix(m, k, seed, stream)
    Q, R = np.linalg.qr(A, mode="reduced")
    return Q * np.sign(np.diag(R))
