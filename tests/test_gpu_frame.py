"""GPU parity of the plain float32 frame kernel against the float64 oracle.

State injection: the oracle's state before frame n is loaded into the GPU
tracker, both process frame n, and y, U, labels, mask and cost values are
compared (tolerances in gpu_common).  Sizes span several workgroup tiles and
a ragged last tile; the 640x480x3 case is the benchmark's launch
configuration."""
import numpy as np
import pytest

from gpu_common import (GUARD, assert_parity, compare_step, f32, oracle_params, oracle_trajectory,
                        say, tracker_kwargs)
from oracle import prost_oracle as O
from synth import video as V

pytestmark = pytest.mark.gpu


def _tracker(prm, storage="f32"):
    import torch
    from paper_1302_2073_amd import Tracker
    assert torch.cuda.is_available()
    return Tracker(prm.width, prm.height, prm.channels, prm.k, **tracker_kwargs(prm, storage))


@pytest.mark.parametrize("frame", [0, 1, 2, 10, 57, 120, 199])
def test_small_gray_step(frame):
    """80x60x1, k = 5: the whole frame fits one workgroup (16 rows per
    thread), so every reduction stays inside it."""
    wl, prm, sv, states = oracle_trajectory("small_gray", 199)
    say(f"small_gray frame {frame}")
    with _tracker(prm) as trk:
        info = trk.launch_info()
        say("  launch", info)
        assert info["workgroups"] == 1
        rep = compare_step(trk, prm, states[frame], f32(sv.frame(frame)))
    assert_parity(rep)


@pytest.mark.parametrize("sync_mode", [0, 1, 2, 3])
@pytest.mark.parametrize("frame", [1, 57])
def test_small_gray_multi_workgroup(frame, sync_mode):
    """The same frames split over a gang of 10 workgroups (one row per
    thread) under each exchange protocol."""
    wl, prm, sv, states = oracle_trajectory("small_gray", 57)
    with _tracker(prm) as trk:
        trk.set_launch(1, sync_mode)
        assert trk.launch_info()["workgroups"] == 10
        rep = compare_step(trk, prm, states[frame], f32(sv.frame(frame)))
    assert_parity(rep)


@pytest.mark.parametrize("frame", [0, 1, 12])
def test_qvga_rgb_step(frame):
    wl, prm, sv, states = oracle_trajectory("qvga_rgb", 12)
    say(f"qvga_rgb frame {frame}")
    with _tracker(prm) as trk:
        say("  launch", trk.launch_info())
        rep = compare_step(trk, prm, states[frame], f32(sv.frame(frame)))
    assert_parity(rep)


@pytest.mark.parametrize("frame", [0, 3])
def test_vga_rgb_step(frame):
    """640x480x3, k=15: the benchmark's workload and launch configuration."""
    wl, prm, sv, states = oracle_trajectory("vga_rgb", 3)
    say(f"vga_rgb frame {frame}")
    with _tracker(prm) as trk:
        say("  launch", trk.launch_info())
        rep = compare_step(trk, prm, states[frame], f32(sv.frame(frame)))
    assert_parity(rep)


def test_vga_rgb_step_at_minimum_step_size():
    """640x480x3, k=15 in the regime n >= i_init of the step-size rule
    (Sec. 3.4: t = t_min): the oracle's state before frame 3 injected with
    frame counter 150, so the geodesic step uses t_min (50x smaller angles
    than at n = 0)."""
    wl, prm, sv, states = oracle_trajectory("vga_rgb", 3)
    st = states[3].copy()
    st.n = 150
    assert O.step_size(150, prm.t_init, prm.t_min, prm.i_init) == prm.t_min
    with _tracker(prm) as trk:
        rep = compare_step(trk, prm, st, f32(sv.frame(3)))
    assert rep["info"].t == prm.t_min
    assert_parity(rep)


@pytest.mark.parametrize("frame", [150, 151])
def test_qvga_rgb_step_after_initialization_phase(frame):
    """320x240x3, k=10 on the oracle's own trajectory past the
    initialization phase (frames 150 and 151 of the jittered video, t =
    t_min): a converged subspace, small angles."""
    wl, prm, sv, states = oracle_trajectory("qvga_rgb", 151)
    with _tracker(prm) as trk:
        rep = compare_step(trk, prm, states[frame], f32(sv.frame(frame)))
    assert rep["info"].t == prm.t_min
    assert_parity(rep)


@pytest.mark.parametrize("curvature", [0, 1])
@pytest.mark.parametrize("cost", ["lp", "log"])
@pytest.mark.parametrize("shape", [(7, 5, 3, 4), (33, 17, 1, 1), (41, 29, 2, 16), (123, 77, 3, 9),
                                   (1, 1, 1, 1), (1, 9, 3, 2), (9, 1, 2, 3), (2, 2, 1, 4)])
def test_random_shapes(shape, cost, curvature):
    """Ragged sizes, k = 1 and k = 16, 1-3 channels, both cost forms, both
    curvature schedules (k = 16: the widest exchange, 153 values).  The
    degenerate frames: one pixel (U = +-1, so the projected gradient and the
    geodesic step vanish), one column or one row of pixels (the median's
    edge clamp on both sides at once), and k = m (U spans the whole space)."""
    W, H, Cc, k = shape
    rank = min(k, 3)
    spec = V.VideoSpec(W, H, Cc, rank=rank, seed=30 + W, noise=0.01, fg_kind="rects",
                       fg_count=2, fg_density=0.1)
    sv = V.SyntheticVideo(spec)
    mu = 1e-3
    prm = O.Params(W, H, Cc, k=k, mu=mu, cost=cost, t_init=5e-3, t_min=1e-4, i_init=20)
    st = O.initial_state(V.initial_subspace(prm.m, k, 3), prm.P)
    for n in range(6):
        st, _ = O.track_frame(st, f32(sv.frame(n)), prm)
    say(f"random shape {shape} cost {cost} curvature {curvature}")
    with _tracker(prm) as trk:
        trk.set_curvature(curvature)
        rep = compare_step(trk, prm, st, f32(sv.frame(6)))
    say(f"  f relative to f_0: {rep['f_rel0']:.1e}")
    assert_parity(rep, f_ref0=(prm.k == prm.m))


def test_labels_before_update_and_filtered_weights():
    wl, prm0, sv, states = oracle_trajectory("small_gray", 30)
    prm = oracle_params(wl, labels_after_update=False, weights_from_filtered=True)
    st = states[30]
    with _tracker(prm) as trk:
        rep = compare_step(trk, prm, st, f32(sv.frame(30)))
    assert_parity(rep)


def test_device_frame_equals_host_frame():
    import torch
    wl, prm, sv, states = oracle_trajectory("small_gray", 20)
    x = sv.frame(20).astype(np.float32)
    st = states[20]
    with _tracker(prm) as trk:
        trk.set_state(st.U, st.y, st.labels, st.n)
        trk.track(x)
        a = trk.get_state()
        ma = trk.mask()
        trk.set_state(st.U, st.y, st.labels, st.n)
        trk.track(torch.from_numpy(x).cuda())
        b = trk.get_state()
        mb = trk.mask()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    assert np.array_equal(ma, mb)


def test_deterministic_bitwise():
    wl, prm, sv, states = oracle_trajectory("qvga_rgb", 2)
    x = sv.frame(2).astype(np.float32)
    outs = []
    with _tracker(prm) as trk:
        for _ in range(3):
            trk.set_state(states[2].U, states[2].y, states[2].labels, 2)
            trk.track(x)
            outs.append(trk.get_state() + (trk.mask(), trk.stats()["f"]))
    for o in outs[1:]:
        for a, b in zip(outs[0][:5], o[:5]):
            assert np.array_equal(a, b)
        assert outs[0][5] == o[5]


def test_degenerate_zero_frame_and_zero_weights():
    """x = 0 with y = 0: zero gradient, CG stops at once, zeta = 0 so U does
    not move; all pixels background.  omega = 0 with every pixel foreground:
    all weights vanish, same outcome."""
    prm = O.Params(20, 10, 3, k=3, mu=1e-3)
    U0 = V.initial_subspace(prm.m, 3, 5)
    st = O.initial_state(U0, prm.P)
    with _tracker(prm) as trk:
        rep = compare_step(trk, prm, st, np.zeros(prm.m))
        assert rep["stats"]["cg_steps"] == 0 and rep["stats"]["updated"] == 0
        assert np.array_equal(rep["U1"], rep["start"].U)
        assert rep["labels"].sum() == 0
    prm0 = O.Params(20, 10, 3, k=3, mu=1e-3, omega=0.0)
    st1 = O.State(U0, np.ones(3) * 0.1, np.ones(prm.P, np.uint8), np.ones(prm.P, np.uint8), 4)
    x = f32(np.random.default_rng(1).random(prm.m))
    with _tracker(prm0) as trk:
        rep = compare_step(trk, prm0, st1, x)
        assert rep["stats"]["cg_steps"] == 0 and rep["stats"]["updated"] == 0
        assert np.array_equal(rep["U1"], rep["start"].U)
    assert_parity(rep)


def test_bad_frame_rejected_state_unchanged():
    import torch
    from paper_1302_2073_amd import _lib as L
    wl, prm, sv, states = oracle_trajectory("small_gray", 5)
    st = states[5]
    x = sv.frame(5).astype(np.float32)
    x[100] = np.nan
    with _tracker(prm) as trk:
        trk.set_state(st.U, st.y, st.labels, st.n)
        before = trk.get_state()
        with pytest.raises(L.ProstError) as ei:
            trk.track(x)                      # host frame: rejected on the host
        assert ei.value.status == L.PROS_EBADFRAME
        xd = torch.from_numpy(x).cuda()
        trk.track(xd)                         # device frame: rejected by the kernel
        assert trk.sync() == L.PROS_EBADFRAME
        after = trk.get_state()
        for a, b in zip(before, after):
            assert np.array_equal(np.asarray(a), np.asarray(b))
        # the tracker keeps working afterwards
        rep = compare_step(trk, prm, st, f32(sv.frame(5)))
    assert_parity(rep)


def test_free_running_small_gray():
    """200 frames on both sides without state injection: report the drift;
    masks disagree on at most 0.5% of pixels per frame."""
    wl, prm, sv, states = oracle_trajectory("small_gray", 199)
    worst = 0.0
    with _tracker(prm) as trk:
        trk.set_state(states[0].U, states[0].y, states[0].labels, 0)
        for n in range(200):
            trk.track(sv.frame(n).astype(np.float32))
            if n + 1 < len(states) and n % 20 == 19:
                U, y, lab, nn = trk.get_state()
                ref = states[n + 1]
                ang = O.principal_angles(ref.U, U).max()
                dis = float(np.mean(lab != ref.labels))
                worst = max(worst, dis)
                say(f"  frame {n}: angle {ang:.2e} y_rel {np.linalg.norm(y - ref.y) / np.linalg.norm(ref.y):.2e} "
                    f"label disagreement {dis:.4%}")
    assert worst <= 0.005


def test_free_running_qvga_rgb_1000_frames():
    """The 320x240x3, k=10 workload (camera jitter, moving ellipses) over its
    1000 frames on both sides from the same U0, no state injection: the
    GPU's labels disagree with the oracle's on at most 0.5% of the pixels
    in every frame; drift of U (largest principal angle) and y reported
    every 100 frames."""
    import time
    from paper_1302_2073_amd import Tracker
    wl = V.qvga_rgb()
    v = wl.video
    prm = oracle_params(wl)
    sv = V.SyntheticVideo(v)
    st = O.initial_state(V.initial_subspace(prm.m, prm.k, v.seed), prm.P)
    worst, worst_n = 0.0, -1
    t0 = time.time()
    with _tracker(prm) as trk:
        trk.set_state(st.U, st.y, st.labels, 0)
        for n in range(wl.n_frames):
            x = sv.frame(n).astype(np.float32)
            st, _ = O.track_frame(st, x.astype(np.float64), prm)
            trk.track(x)
            lab = trk.mask(filtered=False)
            dis = float(np.mean(lab != st.labels))
            if dis > worst:
                worst, worst_n = dis, n
            if n % 100 == 99:
                U, y, _, _ = trk.get_state()
                say(f"  frame {n}: angle {O.principal_angles(st.U, U).max():.2e} "
                    f"y_rel {np.linalg.norm(y - st.y) / np.linalg.norm(st.y):.2e} label disagreement {dis:.4%} "
                    f"({time.time() - t0:.0f} s)")
    say(f"  worst label disagreement {worst:.4%} at frame {worst_n}")
    assert worst <= 0.005


@pytest.mark.parametrize("sync_mode", [0, 1, 2, 3])
@pytest.mark.parametrize("nr", [1, 4, 8])
def test_launch_variants(nr, sync_mode):
    """Register rows per thread (gangs of 452 / 113 / 57 workgroups) and the
    four gang exchanges give the same frame."""
    wl, prm, sv, states = oracle_trajectory("qvga_rgb", 12)
    with _tracker(prm) as trk:
        trk.set_launch(nr, sync_mode)
        say(f"qvga launch {trk.launch_info()}")
        rep = compare_step(trk, prm, states[12], f32(sv.frame(12)))
        assert rep["stats"]["fg_pixels"] == int(rep["labels"].sum())
    assert_parity(rep)


@pytest.mark.parametrize("over", [(("ysolve", "gd"),), (("p", 0.5),), (("p", 1.0),), (("p", 2.0),),
                                  (("ysolve", "gd"), ("p", 1.0)), (("ysolve", "irls"),),
                                  (("ysolve", "irls"), ("p", 1.0)), (("ysolve", "irls"), ("p", 2.0))])
def test_solver_and_exponent_variants(over):
    """Step 1 by gradient descent instead of CG, and p in {0.5, 1, 2} (p = 2:
    a smoothed least-squares tracker), state-injected frames of the 320x240
    workload."""
    wl, prm, sv, states = oracle_trajectory("qvga_rgb", 8, over)
    say(f"qvga variant {dict(over)}")
    with _tracker(prm) as trk:
        rep = compare_step(trk, prm, states[8], f32(sv.frame(8)))
    assert_parity(rep)


@pytest.mark.parametrize("sync_mode", [1, 2, 3])
@pytest.mark.parametrize("nr", [1, 8])
def test_irls_launch_variants(nr, sync_mode):
    """The IRLS step (one wide exchange of g, f and H per step) under each
    tagged exchange and gang size; the counter exchange is refused for it."""
    over = (("ysolve", "irls"),)
    wl, prm, sv, states = oracle_trajectory("qvga_rgb", 8, over)
    with _tracker(prm) as trk:
        with pytest.raises(RuntimeError):
            trk.set_launch(nr, 0)
        trk.set_launch(nr, sync_mode)
        say(f"qvga irls launch {trk.launch_info()}")
        rep = compare_step(trk, prm, states[8], f32(sv.frame(8)))
    assert_parity(rep)


@pytest.mark.parametrize("frame", [0, 3, 40])
def test_irls_small_gray_ragged(frame):
    """IRLS on the small gray workload (a ragged last tile), early frames
    included (t = t_init, few updates behind U)."""
    over = (("ysolve", "irls"),)
    wl, prm, sv, states = oracle_trajectory("small_gray", frame, over)
    with _tracker(prm) as trk:
        rep = compare_step(trk, prm, states[frame], f32(sv.frame(frame)))
    assert_parity(rep)


def _curv_tracker(prm, nr=0, sync_mode=2):
    trk = _tracker(prm)
    if nr or sync_mode != 2:
        trk.set_launch(nr, sync_mode)
    trk.set_curvature(1)
    return trk


@pytest.mark.parametrize("over", [(), (("ysolve", "gd"),), (("p", 1.0),), (("cost", "log"),)])
def test_curvature_schedule_qvga(over):
    """CG with H reduced alongside the gradient (one exchange per step)
    against the oracle, which forms d^T H d from H: 320x240x3, k = 10."""
    wl, prm, sv, states = oracle_trajectory("qvga_rgb", 8, over)
    with _curv_tracker(prm) as trk:
        info = trk.launch_info()
        say(f"qvga curvature 1 {dict(over)} {info}")
        assert info["curvature"] == 1 and info["barriers_per_frame"] == prm.cg_iters + 1
        rep = compare_step(trk, prm, states[8], f32(sv.frame(8)))
    assert_parity(rep)


@pytest.mark.parametrize("sync_mode", [1, 3])
@pytest.mark.parametrize("nr", [1, 4, 8])
def test_curvature_schedule_launch_variants(nr, sync_mode):
    wl, prm, sv, states = oracle_trajectory("qvga_rgb", 12)
    with _curv_tracker(prm, nr, sync_mode) as trk:
        say(f"qvga curvature 1 launch {trk.launch_info()}")
        rep = compare_step(trk, prm, states[12], f32(sv.frame(12)))
    assert_parity(rep)


@pytest.mark.parametrize("frame", [0, 1, 57, 199])
def test_curvature_schedule_small_gray(frame):
    wl, prm, sv, states = oracle_trajectory("small_gray", frame)
    with _curv_tracker(prm) as trk:
        rep = compare_step(trk, prm, states[frame], f32(sv.frame(frame)))
    assert_parity(rep)


def test_curvature_schedule_vga():
    """The benchmark's frame shape, 640x480x3, k = 15 (8 rows per thread)."""
    wl, prm, sv, states = oracle_trajectory("vga_rgb", 3)
    with _curv_tracker(prm) as trk:
        say(f"vga curvature 1 {trk.launch_info()}")
        rep = compare_step(trk, prm, states[3], f32(sv.frame(3)))
    assert_parity(rep)


def test_curvature_schedule_refusals():
    from paper_1302_2073_amd._lib import ProstError
    wl, prm, sv, states = oracle_trajectory("small_gray", 0)
    with _tracker(prm, "bf16") as trk:
        with pytest.raises(ProstError):
            trk.set_curvature(1)
    with _tracker(prm) as trk:
        trk.set_launch(0, 0)
        with pytest.raises(ProstError):
            trk.set_curvature(1)
        trk.set_launch(0, 2)
        trk.set_curvature(1)
        with pytest.raises(ProstError):
            trk.set_launch(0, 0)
        with pytest.raises(ProstError):
            trk.set_curvature(2)
        trk.set_curvature(0)
        assert trk.launch_info()["barriers_per_frame"] == 2 * prm.cg_iters + 1


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_small_gang_automatic_launch(storage):
    """160x120x3 at k = 15 (the resolution Sec. 5.1 tracks at): the automatic
    launch takes a gang of <= 32 workgroups with every workgroup reading all
    partials; parity against the oracle at that launch."""
    spec = V.VideoSpec(160, 120, 3, rank=10, seed=44, noise=0.01, fg_kind="rects", fg_count=3, fg_density=0.05)
    sv = V.SyntheticVideo(spec)
    prm = O.Params(160, 120, 3, k=15, mu=1e-3, t_init=5e-3, t_min=1e-4, i_init=20)
    st = O.initial_state(V.initial_subspace(prm.m, 15, 4), prm.P)
    for n in range(4):
        st, _ = O.track_frame(st, f32(sv.frame(n)), prm)
    with _tracker(prm, storage) as trk:
        info = trk.launch_info()
        say(f"160x120x3 {storage} launch {info}")
        assert info["workgroups"] <= 32 and info["sync_mode"] == 3
        if storage == "f32":
            rep = compare_step(trk, prm, st, f32(sv.frame(4)))
            assert_parity(rep)
        else:
            from test_gpu_precision import _bf16_check, rne_bf16
            _bf16_check(trk, prm, st, rne_bf16(sv.frame(4)), "160x120x3 small gang")


@pytest.mark.parametrize("name,frame", [("qvga_rgb", 8), ("vga_rgb", 3)])
def test_ordinary_dispatch_gives_identical_frames(name, frame):
    """An ordinary launch of the resident grid computes exactly what the
    cooperative launch does (same kernel, same gang), and both match the
    oracle."""
    wl, prm, sv, states = oracle_trajectory(name, frame)
    x = f32(sv.frame(frame)).astype(np.float32)
    outs = []
    for coop in (1, 0):
        with _tracker(prm) as trk:
            trk.set_dispatch(coop)
            trk.set_state(states[frame].U, states[frame].y, states[frame].labels, states[frame].n)
            trk.track(x)
            trk.track(x)
            outs.append(trk.get_state())
            assert trk.sync() == 0
    for a, b in zip(outs[0], outs[1]):
        np.testing.assert_array_equal(a, b)
    with _tracker(prm) as trk:
        trk.set_dispatch(0)
        rep = compare_step(trk, prm, states[frame], f32(sv.frame(frame)))
    assert_parity(rep)
