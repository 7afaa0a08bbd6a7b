"""GPU parity of the Sec. 3.4 pre-processing (running average of the
initialization frames subtracted, scaled by their pooled standard
deviation), in the single-stream kernels (both storage types) and in the
batched form, against the float64 oracle."""
import numpy as np
import pytest

from gpu_common import (GUARD, assert_parity, compare_step, f32, oracle_trajectory, say, tracker_kwargs,
                        update_rounding_bound)
from oracle import prost_oracle as O
from synth import video as V

pytestmark = pytest.mark.gpu

OVER = (("preprocess", True), ("i_init", 10))


def _tracker(prm, storage="f32"):
    from paper_1302_2073_amd import Tracker
    return Tracker(prm.width, prm.height, prm.channels, prm.k, **tracker_kwargs(prm, storage))


@pytest.mark.parametrize("frame", [0, 1, 2, 5, 9, 10, 14])
def test_small_gray_preprocessed_step(frame):
    """Frame 0 (all zero after mean removal), frames inside the
    initialization phase (statistics updated) and after it (frozen)."""
    wl, prm, sv, states = oracle_trajectory("small_gray", 14, OVER)
    say(f"small_gray pre-processed frame {frame}")
    with _tracker(prm) as trk:
        rep = compare_step(trk, prm, states[frame], f32(sv.frame(frame)))
        if frame == 0:
            assert rep["stats"]["updated"] == 0
    assert_parity(rep)


@pytest.mark.parametrize("frame", [2, 6])
def test_qvga_preprocessed_step(frame):
    wl, prm, sv, states = oracle_trajectory("qvga_rgb", 6, (("preprocess", True), ("i_init", 4)))
    with _tracker(prm) as trk:
        rep = compare_step(trk, prm, states[frame], f32(sv.frame(frame)))
    assert_parity(rep)


def _rne(a):
    f = np.asarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    return ((((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32)).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("frame", [3, 12])
def test_bf16_preprocessed_step(frame):
    wl, prm, sv, states = oracle_trajectory("small_gray", 14, OVER)
    x = _rne(sv.frame(frame))
    with _tracker(prm, "bf16") as trk:
        rep = compare_step(trk, prm, states[frame], x, storage="bf16")
    exp = _rne(rep["exp"].U)
    ulp = np.exp2(np.floor(np.log2(np.maximum(np.abs(exp), 1e-38))) - 7)
    ulp = ulp + update_rounding_bound(rep["start"], x, prm, rep["exp"].y, rep["y1"])
    over = int(np.sum(np.abs(rep["U1"] - exp) > ulp * (1 + 1e-12)))
    say(f"  bf16 pre-processed frame {frame}: y {rep['y_rel']:.1e} U beyond bound {over} pre {rep['pre']}")
    assert rep["y_rel"] <= 1e-4 and over == 0 and rep["lab_mismatch_outside_band"] == 0
    assert rep["pre"]["count"][0] == rep["pre"]["count"][1]
    assert rep["pre"]["mean_err"] <= 1e-6 and rep["pre"]["m2_rel"] <= 1e-4


def test_batch_preprocessed_streams_follow_the_oracle():
    """Two streams with pre-processing in one batch, frames 0..5 across the
    end of a 4-frame initialization phase, each step against the oracle
    step from the device's own state and statistics: y and U within 1e-4,
    labels exact outside the guard band."""
    import torch
    from paper_1302_2073_amd.tracker import BatchTracker
    shapes = [(48, 32, 1, 4), (40, 30, 3, 6)]
    streams = []
    for i, (W, H, Cc, k) in enumerate(shapes):
        spec = V.VideoSpec(W, H, Cc, rank=3, seed=70, stream=i, noise=0.01, fg_kind="rects", fg_count=2,
                           fg_density=0.1)
        prm = O.Params(W, H, Cc, k=k, mu=1e-3, i_init=4, preprocess=True)
        U0 = V.initial_subspace(prm.m, k, 70, i)
        streams.append((V.SyntheticVideo(spec), prm, U0))
    specs = [dict(width=p.width, height=p.height, channels=p.channels, k=p.k, mu=p.mu, i_init=p.i_init,
                  preprocess=True) for _, p, _ in streams]
    with BatchTracker(specs) as bt:
        frames = [[torch.from_numpy(sv.frame(n).astype(np.float32)).cuda() for n in range(6)]
                  for sv, _, _ in streams]
        bt.set_frames(frames)
        for s, (sv, prm, U0) in enumerate(streams):
            bt.set_state(s, U0)
        for n in range(6):
            exp = []
            for s, (sv, prm, U0) in enumerate(streams):   # the oracle step from the device's state
                U0d, y0d, l0d, n0d = bt.get_state(s)
                mean_d, m2_d, cnt_d, _ = bt.get_preprocess(s)
                pre = O.Preproc(mean_d * cnt_d, m2_d + mean_d * mean_d * cnt_d, cnt_d)
                start = O.State(U0d, y0d, l0d, O.median3x3(l0d, prm.height, prm.width), n0d, pre)
                exp.append(O.track_frame(start, f32(sv.frame(n)), prm))
            bt.step()
            assert bt.sync() == 0
            for s, (sv, prm, U0) in enumerate(streams):
                ref, info = exp[s]
                U1, y1, l1, n1 = bt.get_state(s)
                y_rel = np.linalg.norm(y1 - ref.y) / max(np.linalg.norm(ref.y), 1e-30)
                U_rel = np.linalg.norm(U1 - ref.U) / np.linalg.norm(ref.U)
                band = O.band_pixels(ref.U, info.x, ref.y, prm.thr, prm.channels, GUARD)
                outside = int(np.sum((l1 != ref.labels) & ~band))
                say(f"  frame {n} stream {s}: y {y_rel:.1e} U {U_rel:.1e} labels differ "
                    f"{int(np.sum(l1 != ref.labels))} (outside the band {outside}, band {int(band.sum())})")
                assert n1 == ref.n
                assert (y_rel <= 1e-4 or np.linalg.norm(ref.y) < 1e-12) and U_rel <= 1e-4
                assert outside == 0
