"""The largest frame whose register tiles stay on chip, and the streamed
form beyond it.

Every workgroup of a stream's gang keeps its tile of U in registers for the
whole frame, so the gang must be resident at once: pros_init takes the
widest tile built for (storage, k) for frames up to that size, and the
streamed form (one launch per dependent pass, U read from HBM in every
pass) for larger ones.  The boundary is found by bisection over the frame
height (width 640, three colour channels, k = 15); one frame at the largest
resident size and frames of the streamed form (one row beyond it, a
1280x720x3 frame at k = 15, small ragged frames forced into the streamed
form) are checked against the float64 oracle."""
import numpy as np
import pytest

from gpu_common import TOL_STEP, TOL_Y, assert_parity, compare_step, f32, oracle_params, say, tracker_kwargs
from oracle import prost_oracle as O
from synth import video as V

pytestmark = pytest.mark.gpu

WIDTH, CH, K = 640, 3, 15


def _spec(height):
    v = V.VideoSpec(WIDTH, height, CH, rank=10, seed=5, noise=0.01, fg_kind="rects", fg_count=3,
                    fg_density=0.05, speed=(1.0, 2.0))
    return O.Params(WIDTH, height, CH, k=K, mu=1e-3), v


def _accepts(height, storage):
    """Launch of a frame of this height when its tiles stay on chip, None
    when it runs the streamed form."""
    from paper_1302_2073_amd import Tracker
    prm, _ = _spec(height)
    with Tracker(WIDTH, height, CH, K, **tracker_kwargs(prm, storage)) as trk:
        info = trk.launch_info()
    return None if info["sync_mode"] == -1 else info


def _largest(storage):
    lo, hi = 480, 8192       # 640x480x3 at k = 15 is accepted; 640x8192x3 is not
    assert _accepts(lo, storage) is not None and _accepts(hi, storage) is None
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if _accepts(mid, storage) is not None:
            lo = mid
        else:
            hi = mid
    return lo


def _start_state(prm, v, frames):
    sv = V.SyntheticVideo(v)
    st = O.initial_state(V.initial_subspace(prm.m, prm.k, v.seed), prm.P)
    for n in range(frames):
        st, _ = O.track_frame(st, f32(sv.frame(n)), prm)
    return sv, st


def test_largest_float32_frame_matches_the_oracle():
    import torch
    H = _largest("f32")
    info = _accepts(H, "f32")
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    say(f"float32: largest 640x{H}x3 at k = 15, launch {info}, {cus} CUs")
    # one row of pixels more needs one workgroup beyond what can be resident
    assert info["workgroups"] * info["pixels_per_wg"] < WIDTH * (H + 1)
    prm, v = _spec(H)
    sv, st = _start_state(prm, v, 1)
    from paper_1302_2073_amd import Tracker
    with Tracker(WIDTH, H, CH, K, **tracker_kwargs(prm, "f32")) as trk:
        rep = compare_step(trk, prm, st, f32(sv.frame(1)))
    assert_parity(rep)


def test_largest_bfloat16_frame_matches_the_oracle():
    from test_gpu_precision import _bf16_check, rne_bf16
    H = _largest("bf16")
    info = _accepts(H, "bf16")
    say(f"bfloat16: largest 640x{H}x3 at k = 15, launch {info}")
    assert H > _largest("f32")     # two rows per register: a larger frame fits
    prm, v = _spec(H)
    sv, st = _start_state(prm, v, 1)
    from paper_1302_2073_amd import Tracker
    with Tracker(WIDTH, H, CH, K, **tracker_kwargs(prm, "bf16")) as trk:
        _bf16_check(trk, prm, st, rne_bf16(sv.frame(1)), f"640x{H}x3")


def _streamed_step(prm, st, x64, storage="f32", force=False, curvature=0):
    from paper_1302_2073_amd import Tracker
    with Tracker(prm.width, prm.height, prm.channels, prm.k, **tracker_kwargs(prm, storage)) as trk:
        if force:
            trk.set_launch(-1)
        trk.set_curvature(curvature)
        info = trk.launch_info()
        assert info["sync_mode"] == -1, info
        say(f"  streamed {prm.width}x{prm.height}x{prm.channels} k={prm.k}: {info}")
        return compare_step(trk, prm, st, x64, storage=storage)


def test_one_row_beyond_the_resident_size_is_streamed():
    H = _largest("f32") + 1
    prm, v = _spec(H)
    sv, st = _start_state(prm, v, 1)
    rep = _streamed_step(prm, st, f32(sv.frame(1)))
    assert_parity(rep)


@pytest.mark.parametrize("n,curvature", [(0, 0), (150, 0), (150, 1)])
def test_streamed_1280x720_float32(n, curvature):
    """1280x720x3 at k = 15 (four times the 640x480 frame, beyond the
    resident register tiles) against the oracle, before and after the
    initialization phase of the step-size rule, with either curvature
    schedule of the CG step."""
    spec = V.VideoSpec(1280, 720, 3, rank=10, seed=7, noise=0.01, fg_kind="rects", fg_count=3, fg_density=0.05,
                       speed=(1.0, 2.0))
    prm = O.Params(1280, 720, 3, k=15, mu=1e-3)
    sv, st = _start_state(prm, spec, 1)
    st.n = n
    rep = _streamed_step(prm, st, f32(sv.frame(1)), curvature=curvature)
    assert_parity(rep)


def test_streamed_1280x720_bfloat16():
    from test_gpu_precision import _bf16_check, rne_bf16
    from paper_1302_2073_amd import Tracker
    spec = V.VideoSpec(1280, 720, 3, rank=10, seed=8, noise=0.01, fg_kind="rects", fg_count=3, fg_density=0.05,
                       speed=(1.0, 2.0))
    prm = O.Params(1280, 720, 3, k=15, mu=1e-3)
    sv = V.SyntheticVideo(spec)
    st = O.initial_state(rne_bf16(V.initial_subspace(prm.m, prm.k, spec.seed)), prm.P)
    st, _ = O.track_frame(st, rne_bf16(sv.frame(0)), prm)
    with Tracker(1280, 720, 3, 15, **tracker_kwargs(prm, "bf16")) as trk:
        info = trk.launch_info()
        say(f"  bfloat16 1280x720x3 launch {info}")
        # bfloat16 pair tiles hold twice the rows: 1280x720x3 still needs the streamed form
        assert info["sync_mode"] == -1
        _bf16_check(trk, prm, st, rne_bf16(sv.frame(1)), "1280x720x3 streamed")


@pytest.mark.parametrize("cost", ["lp", "log"])
@pytest.mark.parametrize("shape", [(7, 5, 3, 4), (33, 17, 1, 1), (123, 77, 3, 9), (41, 29, 2, 16), (1, 9, 3, 2)])
@pytest.mark.parametrize("curvature", [0, 1])
def test_streamed_form_on_small_frames(shape, cost, curvature):
    """The streamed form forced on small ragged frames (partial last
    workgroup, k = 1 and k = 16, 1-3 channels, both cost forms, both
    curvature schedules) against the oracle."""
    W, H, Cc, k = shape
    spec = V.VideoSpec(W, H, Cc, rank=min(k, 3), seed=90 + W, noise=0.01, fg_kind="rects", fg_count=2,
                       fg_density=0.1)
    sv = V.SyntheticVideo(spec)
    prm = O.Params(W, H, Cc, k=k, mu=1e-3, cost=cost, t_init=5e-3, t_min=1e-4, i_init=20)
    st = O.initial_state(V.initial_subspace(prm.m, k, 3), prm.P)
    for n in range(6):
        st, _ = O.track_frame(st, f32(sv.frame(n)), prm)
    rep = _streamed_step(prm, st, f32(sv.frame(6)), force=True, curvature=curvature)
    from paper_1302_2073_amd import Tracker
    with Tracker(W, H, Cc, k, **tracker_kwargs(prm)) as trk:   # the register-tile kernel on the same frame
        tiles = compare_step(trk, prm, st, f32(sv.frame(6)))
    say(f"  register tiles: y_rel={tiles['y_rel']:.2e} theta_rel={tiles['theta_rel']:.1e} "
        f"alpha_rel={tiles['alpha_rel']:.1e}")
    # A frame of a few dozen entries can make the CG steps ill-conditioned:
    # the bound there is four times the oracle's own spread when x moves by
    # one float32 ulp (the rounding of a float32 residual), if that is larger.
    sy, ss = _input_sensitivity(prm, st, f32(sv.frame(6)))
    say(f"  oracle spread at one ulp of x: y {sy:.1e} theta/alpha {ss:.1e}")
    assert_parity(rep, tol_y=max(TOL_Y, 4 * sy), tol_step=max(TOL_STEP, 4 * ss))


def _input_sensitivity(prm, st, x, trials=8):
    """Largest relative change of y, theta and the CG steps alpha of one
    oracle frame when every entry of x is scaled by (1 + 2^-24 z), z ~ N(0, 1),
    from the state with U rounded to float32."""
    start = O.State(f32(st.U), st.y, st.labels, O.median3x3(st.labels, prm.height, prm.width), st.n, st.pre)
    ref, info = O.track_frame(start, x, prm)
    rng = np.random.default_rng(1)
    sy = ss = 0.0
    for _ in range(trials):
        e, i2 = O.track_frame(start, x * (1.0 + 2.0 ** -24 * rng.standard_normal(x.shape)), prm)
        sy = max(sy, float(np.linalg.norm(e.y - ref.y) / np.linalg.norm(ref.y)))
        ss = max(ss, abs(i2.theta - info.theta) / abs(info.theta))
        for a0, a1 in zip(info.cg.alpha, i2.cg.alpha):
            ss = max(ss, abs(a1 - a0) / abs(a0))
    return sy, ss


def test_streamed_free_running_matches_tiles():
    """The 80x60 workload over 60 frames in the streamed form beside the
    oracle from the same U0: labels agree on at least 99.5% of the pixels in
    every frame; a rejected (non-finite) frame leaves the state unchanged."""
    from paper_1302_2073_amd import Tracker
    from paper_1302_2073_amd import _lib as L
    wl = V.small_gray()
    prm = oracle_params(wl)
    sv = V.SyntheticVideo(wl.video)
    st = O.initial_state(V.initial_subspace(prm.m, prm.k, wl.video.seed), prm.P)
    worst = 0.0
    with Tracker(80, 60, 1, wl.k, **tracker_kwargs(prm)) as trk:
        trk.set_launch(-1)
        trk.set_state(st.U, st.y, st.labels, 0)
        for n in range(60):
            x = sv.frame(n).astype(np.float32)
            st, _ = O.track_frame(st, x.astype(np.float64), prm)
            trk.track(x)
            worst = max(worst, float(np.mean(trk.mask(filtered=False) != st.labels)))
        U0, y0, l0, n0 = trk.get_state()
        bad = sv.frame(60).astype(np.float32)
        bad[17] = np.nan
        with pytest.raises(L.ProstError):   # rejected by the host check of a host frame
            trk.track(bad)
        import torch
        trk.track(torch.from_numpy(bad).cuda())   # a device frame is checked on the device
        assert trk.sync() == L.PROS_EBADFRAME
        U1, y1, l1, n1 = trk.get_state()
        assert n1 == n0 and np.array_equal(U1, U0) and np.array_equal(y1, y0) and np.array_equal(l1, l0)
    say(f"  worst label disagreement over 60 streamed frames: {worst:.4%}")
    assert worst <= 0.005


@pytest.mark.parametrize("shape", [(40, 30, 3, 15), (33, 17, 1, 4), (64, 47, 2, 16)])
@pytest.mark.parametrize("curvature", [0, 1])
def test_streamed_bfloat16_small_frames(shape, curvature):
    """The streamed form in bfloat16 storage, forced on small frames: even P
    (two adjacent pixels per thread, 32-bit accesses) and odd P (one pixel
    per thread), both curvature schedules, against the oracle on bfloat16
    inputs."""
    from test_gpu_precision import _bf16_check, rne_bf16
    from paper_1302_2073_amd import Tracker
    W, H, Cc, k = shape
    spec = V.VideoSpec(W, H, Cc, rank=min(k, 3), seed=70 + W, noise=0.01, fg_kind="rects", fg_count=2,
                       fg_density=0.1)
    sv = V.SyntheticVideo(spec)
    prm = O.Params(W, H, Cc, k=k, mu=1e-3, t_init=5e-3, t_min=1e-4, i_init=20)
    st = O.initial_state(rne_bf16(V.initial_subspace(prm.m, k, 5)), prm.P)
    for n in range(4):
        st, _ = O.track_frame(st, rne_bf16(sv.frame(n)), prm)
    with Tracker(W, H, Cc, k, **tracker_kwargs(prm, "bf16")) as trk:
        trk.set_launch(-1)
        trk.set_curvature(curvature)
        assert trk.launch_info()["sync_mode"] == -1
        _bf16_check(trk, prm, st, rne_bf16(sv.frame(4)), f"{W}x{H}x{Cc} k={k} streamed, schedule {curvature}")


def test_streamed_bfloat16_device_frames_at_both_alignments():
    """A bfloat16 device frame of the streamed form at a 4-byte aligned
    address (pixel pairs) and at an odd element offset (one pixel per
    thread): both steps follow the oracle (y within 1e-4, labels exact
    outside the guard band) from the same injected state."""
    import torch
    from test_gpu_precision import rne_bf16
    from paper_1302_2073_amd import Tracker
    from paper_1302_2073_amd.tracker import bf16_bits
    from gpu_common import GUARD
    W, H, Cc, k = 64, 48, 3, 10
    spec = V.VideoSpec(W, H, Cc, rank=3, seed=71, noise=0.01, fg_kind="rects", fg_count=2, fg_density=0.1)
    sv = V.SyntheticVideo(spec)
    prm = O.Params(W, H, Cc, k=k, mu=1e-3, i_init=20)
    st = O.initial_state(rne_bf16(V.initial_subspace(prm.m, k, 6)), prm.P)
    for n in range(3):
        st, _ = O.track_frame(st, rne_bf16(sv.frame(n)), prm)
    x64 = rne_bf16(sv.frame(3))
    x = torch.from_numpy(bf16_bits(x64).view(np.int16)).cuda().view(torch.bfloat16)
    for offset in (0, 1):
        with Tracker(W, H, Cc, k, **tracker_kwargs(prm, "bf16")) as trk:
            trk.set_launch(-1)
            trk.set_state(st.U, st.y, st.labels, st.n)
            U0, y0, l0, n0 = trk.get_state()
            start = O.State(U0, y0, l0, O.median3x3(l0, prm.height, prm.width), n0)
            exp, _ = O.track_frame(start, x64, prm)
            buf = torch.empty(prm.m + 1, dtype=torch.bfloat16, device="cuda")
            view = buf[offset:offset + prm.m]
            view.copy_(x)
            torch.cuda.synchronize()
            trk.track(view)
            assert trk.sync() == 0
            U1, y1, l1, n1 = trk.get_state()
        band = O.band_pixels(exp.U, x64, exp.y, prm.thr, prm.channels, GUARD)
        y_rel = np.linalg.norm(y1 - exp.y) / np.linalg.norm(exp.y)
        say(f"  offset {offset}: y_rel {y_rel:.2e}, labels outside band {int(np.sum((l1 != exp.labels) & ~band))}")
        assert n1 == exp.n and y_rel <= TOL_Y
        assert int(np.sum((l1 != exp.labels) & ~band)) == 0
