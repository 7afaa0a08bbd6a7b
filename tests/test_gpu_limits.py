"""The largest frame one stream accepts, and the first size it refuses.

Every workgroup of a stream's gang keeps its tile of U in registers for the
whole frame, so the gang must be resident at once: pros_init takes the
widest tile built for (storage, k) and refuses, with PROS_EUNSUPPORTED and
before any launch, a frame that needs more workgroups than the device keeps
resident.  The boundary is found by bisection over the frame height (width
640, three colour channels, k = 15), and one frame at the largest accepted
size is checked against the float64 oracle."""
import numpy as np
import pytest

from gpu_common import assert_parity, compare_step, f32, say, tracker_kwargs
from oracle import prost_oracle as O
from synth import video as V

pytestmark = pytest.mark.gpu

WIDTH, CH, K = 640, 3, 15


def _spec(height):
    v = V.VideoSpec(WIDTH, height, CH, rank=10, seed=5, noise=0.01, fg_kind="rects", fg_count=3,
                    fg_density=0.05, speed=(1.0, 2.0))
    return O.Params(WIDTH, height, CH, k=K, mu=1e-3), v


def _accepts(height, storage):
    from paper_1302_2073_amd import Tracker
    from paper_1302_2073_amd import _lib as L
    prm, _ = _spec(height)
    try:
        with Tracker(WIDTH, height, CH, K, **tracker_kwargs(prm, storage)) as trk:
            return trk.launch_info()
    except L.ProstError as e:
        assert e.status == L.PROS_EUNSUPPORTED, str(e)
        assert "does not fit" in str(e)
        return None


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
