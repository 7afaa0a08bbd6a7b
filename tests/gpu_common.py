"""Shared helpers of the GPU parity tests: oracle trajectories on the same
seeded inputs, state injection, comparison at the stated tolerances."""
import functools
import sys

import numpy as np

from oracle import prost_oracle as O
from synth import video as V

# Parity bar (per state-injected frame, float32 kernels vs the float64 oracle)
TOL_Y = 1e-4          # ||y - y*|| / ||y*||
TOL_U = 1e-4          # ||U - U*||_F / ||U*||_F
GUARD = 1e-5          # labels compared exactly where | max_c |r'| - delta | > GUARD
TOL_F = 1e-5          # cost values, relative
TOL_STEP = 1e-5       # geodesic angle theta and CG step lengths alpha, relative
TOL_U_ELEM = 1e-5     # max_e,j |U - U*| / max |U*| (float32 storage)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def oracle_params(wl, **over):
    v = wl.video
    kw = dict(k=wl.k, mu=wl.mu, delta=wl.delta, cost=wl.cost)
    kw.update(over)
    return O.Params(v.width, v.height, v.channels, **kw)


def tracker_kwargs(prm: O.Params, storage="f32"):
    return dict(cg_iters=prm.cg_iters, cost=prm.cost, p=prm.p, mu=prm.mu, delta=prm.delta,
                omega=prm.omega, t_init=prm.t_init, t_min=prm.t_min, i_init=prm.i_init,
                storage=storage, labels_after_update=prm.labels_after_update,
                weights_from_filtered=prm.weights_from_filtered, preprocess=prm.preprocess, ysolve=prm.ysolve)


@functools.lru_cache(maxsize=8)
def oracle_trajectory(name, upto, over_items=()):
    """Oracle states before frames 0..upto of a named workload, on float32
    frames (the kernels' input)."""
    wl = WORKLOADS[name]()
    prm = oracle_params(wl, **dict(over_items))
    sv = V.SyntheticVideo(wl.video)
    st = O.initial_state(V.initial_subspace(prm.m, prm.k, wl.video.seed), prm.P)
    states = []
    for n in range(upto + 1):
        states.append(st.copy())
        st, _ = O.track_frame(st, f32(sv.frame(n)), prm)
    return wl, prm, sv, states


WORKLOADS = {
    "small_gray": V.small_gray,
    "qvga_rgb": V.qvga_rgb,
    "vga_rgb": V.vga_rgb,
}


def compare_step(trk, prm, st, x64, storage="f32", guard=GUARD):
    """Inject oracle state `st`, run one frame on the GPU and on the oracle
    (from the state as rounded by the device), return a report dict."""
    trk.set_state(st.U, st.y, st.labels, st.n)
    U0, y0, l0, n0 = trk.get_state()
    pre_dev = None
    if prm.preprocess:   # inject the statistics and continue from their float32 copy
        pre = st.pre if st.pre is not None else O.preproc_init(prm.m)
        trk.set_preprocess(pre.mean, pre.m2, pre.count)
        mean_d, m2_d, cnt_d, _ = trk.get_preprocess()
        pre_dev = O.Preproc(mean_d * cnt_d, m2_d + mean_d * mean_d * cnt_d, cnt_d)
    # the kernel filters the injected labels at the start of the frame, as
    # the oracle's state after a frame holds the median of its labels
    start = O.State(U0, y0, l0, O.median3x3(l0, prm.height, prm.width), n0, pre_dev)
    exp, info = O.track_frame(start, x64, prm)
    if storage == "f32":
        trk.track(x64.astype(np.float32))
    else:
        from paper_1302_2073_amd.tracker import bf16_bits
        trk.track(bf16_bits(x64))
    U1, y1, l1, n1 = trk.get_state()
    mask = trk.mask(filtered=True)
    stats = trk.stats()
    U_lab = exp.U if prm.labels_after_update else start.U
    xs = info.x if info.x is not None else x64      # the frame the steps ran on
    band = O.band_pixels(U_lab, xs, exp.y, prm.thr, prm.channels, guard)
    rep = dict(
        n=n1, n_exp=exp.n,
        y_rel=float(np.linalg.norm(y1 - exp.y) / max(np.linalg.norm(exp.y), 1e-300)),
        U_rel=float(np.linalg.norm(U1 - exp.U) / np.linalg.norm(exp.U)),
        lab_mismatch_outside_band=int(np.sum((l1 != exp.labels) & ~band)),
        band=int(band.sum()),
        lab_mismatch=int(np.sum(l1 != exp.labels)),
        mask_vs_median_of_gpu_labels=int(np.sum(mask != O.median3x3(l1, prm.height, prm.width))),
        f_rel=float(max(abs(a - b) / max(abs(b), 1e-300) for a, b in zip(stats["f"], info.cg.f))) if stats["f"] else 0.0,
        f_rel0=float(max(abs(a - b) for a, b in zip(stats["f"], info.cg.f)) / max(abs(info.cg.f[0]), 1e-300))
        if stats["f"] else 0.0,
        theta_rel=float(abs(stats["theta"] - info.theta) / max(abs(info.theta), 1e-300)),
        # step lengths of the steps that matter: those that decrease the cost by
        # at least 0.1% of the frame's whole decrease (near an exact fit a
        # step's gradient is at rounding level and its length ill-conditioned,
        # while the step itself is negligible)
        alpha_rel=float(max([abs(a - b) / max(abs(b), 1e-300)
                             for j, (a, b) in enumerate(zip(stats["alpha"], info.cg.alpha))
                             if info.cg.f[j] - info.cg.f[j + 1] >= 1e-3 * (info.cg.f[0] - info.cg.f[-1])]
                            + [0.0])),
        U_elem=float(np.max(np.abs(U1 - exp.U)) / np.max(np.abs(exp.U))),
        steps=(stats["cg_steps"], info.cg.iters),
        cg_iters=prm.cg_iters,
        U1=U1, exp=exp, info=info, stats=stats, y1=y1, labels=l1, mask=mask, start=start,
    )
    if prm.preprocess:
        mean1, m21, cnt1, _ = trk.get_preprocess()
        em, ev = exp.pre.mean, exp.pre.m2
        rep["pre"] = dict(count=(cnt1, exp.pre.count),
                          mean_err=float(np.max(np.abs(mean1 - em)) / max(np.max(np.abs(em)), 1e-30)),
                          m2_rel=float(np.linalg.norm(m21 - ev) / max(np.linalg.norm(ev), 1e-30)))
    return rep


def assert_parity(rep, tol_y=TOL_Y, tol_u=TOL_U, f_ref0=False, tol_step=TOL_STEP):
    """f_ref0: compare the costs relative to the frame's first cost f_0
    instead of each f_j.  For frames the subspace fits exactly (k = m) the
    log cost's f_j tends to 0, and the float32 residuals (absolute error
    about 2^-24 |x|) then leave a large relative error on f_j alone."""
    say(f"  n={rep['n']} y_rel={rep['y_rel']:.2e} U_rel={rep['U_rel']:.2e} U_elem={rep['U_elem']:.2e} "
        f"band={rep['band']} lab_mism={rep['lab_mismatch']} outside={rep['lab_mismatch_outside_band']} "
        f"f_rel={rep['f_rel']:.1e} theta_rel={rep['theta_rel']:.1e} alpha_rel={rep['alpha_rel']:.1e} "
        f"steps={rep['steps']}")
    assert rep["n"] == rep["n_exp"]
    dev_steps, ora_steps = rep["steps"]
    if ora_steps < rep["cg_iters"]:
        # The oracle stopped early at an exactly zero gradient or curvature
        # (the exact minimiser, e.g. a one-pixel frame with k = 1).  Whether
        # g is exactly zero is a floating-point decision: the kernel's
        # float32 residual leaves g at rounding level, so it may take further
        # steps, which must leave y within the tolerance.
        assert ora_steps <= dev_steps <= rep["cg_iters"]
    else:
        assert dev_steps == ora_steps
    assert rep["y_rel"] <= tol_y
    assert rep["U_rel"] <= tol_u
    assert rep["lab_mismatch_outside_band"] == 0
    assert rep["mask_vs_median_of_gpu_labels"] == 0
    assert (rep["f_rel0"] if f_ref0 else rep["f_rel"]) <= TOL_F
    assert rep["U_elem"] <= TOL_U_ELEM
    if not f_ref0:   # (an exactly fitted frame drives theta and the last alpha to rounding level)
        assert rep["theta_rel"] <= tol_step
        assert rep["alpha_rel"] <= tol_step
    if "pre" in rep:   # float32 running statistics against float64
        say(f"  pre-processing: count {rep['pre']['count']} mean {rep['pre']['mean_err']:.1e} "
            f"m2 {rep['pre']['m2_rel']:.1e}")
        assert rep["pre"]["count"][0] == rep["pre"]["count"][1]
        assert rep["pre"]["mean_err"] <= 1e-6 and rep["pre"]["m2_rel"] <= 1e-4


def update_rounding_bound(start, x64, prm, y_final, y_dev=None):
    """Per-entry bound of the float32 error of the geodesic update
    u' = u + [(cos(theta)-1) (u.v) - (sin(theta)/zeta) (eta - u.a)] v, from the
    oracle's float64 intermediates:
    * 2^-20 times the magnitudes of the terms (a float32 error of a few units
      in the last place of each of them);
    * the residual's own float32 error and the device's y (y_dev, which the
      parity bar allows to differ from the oracle's), carried into eta by
      the cost's second derivative (largest at r = 0) and into v = y/||y||."""
    import math
    U = start.U
    x_err = 0.0
    if prm.preprocess:   # the steps run on the pre-processed frame, itself rounded to float32
        pre = start.pre if start.pre is not None else O.preproc_init(prm.m)
        scale = O.preproc_scale(pre)
        x64, pre2 = O.preprocess(pre, x64, start.n, prm.i_init)
        x_err = 2.0 ** -21 * (np.abs(x64) + np.abs(pre2.mean) / scale)
    w = O.pixel_weights(start.mask if prm.weights_from_filtered else start.labels, prm.omega, prm.channels)
    eta = O.eta_vector(U, x64, y_final, w, prm.p, prm.mu, prm.cost)
    s, sigma, v, zeta, nu = O.rank_one_svd(U, eta, y_final)
    if s is None or v is None:
        return 2.0 ** -20 * np.abs(U)
    theta = sigma * O.step_size(start.n, prm.t_init, prm.t_min, prm.i_init)
    a = U.T @ eta
    term = (abs(math.cos(theta) - 1.0) * np.abs(U @ v) + abs(math.sin(theta) / zeta) * (np.abs(eta) + np.abs(U @ a)))
    bound = 2.0 ** -20 * (np.abs(U) + np.abs(term)[:, None] * np.abs(v)[None, :])
    dy = 0.0 if y_dev is None else float(np.linalg.norm(np.asarray(y_dev) - y_final))
    dr = 2.0 ** -20 * (np.abs(x64) + np.abs(U) @ np.abs(y_final)) + np.linalg.norm(U, axis=1) * dy + x_err
    if prm.cost == "log":
        phi2 = 2.0 / prm.mu
    else:
        phi2 = prm.p * prm.mu ** (prm.p / 2.0 - 1.0)
    deta = w * phi2 * dr
    bound += abs(math.sin(theta) / zeta) * deta[:, None] * np.abs(v)[None, :]
    bound += np.abs(term)[:, None] * (dy / nu)
    return bound
