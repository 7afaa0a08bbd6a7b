"""Sequence launches (pros_track_frames): several frames per launch of the
persistent kernel, the U tile kept in registers between them.  The result
must equal one pros_track_frame per frame bit for bit (same arithmetic on the
same values), under every exchange protocol, with a rejected frame inside
the sequence and with re-orthonormalisation splitting it."""
import numpy as np
import pytest

from gpu_common import f32, say
from synth import video as V

pytestmark = pytest.mark.gpu


def _frames(wl, n, storage, bad=None):
    import torch
    from paper_1302_2073_amd.tracker import bf16_bits
    sv = V.SyntheticVideo(wl.video)
    out = []
    for i in range(n):
        x = f32(sv.frame(i)).astype(np.float32)
        if bad is not None and i == bad:
            x = x.copy()
            x[7] = np.nan
        if storage == "bf16":
            out.append(torch.from_numpy(bf16_bits(x).view(np.int16)).cuda().view(torch.bfloat16))
        else:
            out.append(torch.from_numpy(x).cuda())
    return out


def _run(wl, frames, storage, seq, nr=0, mode=2, coop=1, **kw):
    from paper_1302_2073_amd import Tracker
    v = wl.video
    with Tracker(v.width, v.height, v.channels, wl.k, mu=wl.mu, delta=wl.delta, cost=wl.cost, storage=storage,
                 **kw) as trk:
        if nr:
            trk.set_launch(nr, mode)
        trk.set_dispatch(coop)
        trk.set_state(V.initial_subspace(trk.m, wl.k, 3))
        if seq:
            trk.track_many(frames)
        else:
            for f in frames:
                trk.track(f)
        st = trk.sync()
        state = trk.get_state()
        stats = trk.stats()
        mask = trk.mask()
        info = trk.launch_info()
    return st, state, stats, mask, info


def _same(a, b):
    assert a[0] == b[0]
    for x, y in zip(a[1], b[1]):
        np.testing.assert_array_equal(x, y)
    for key in ("frame", "cg_steps", "restarts", "updated", "bad_frame", "f", "alpha", "beta", "theta", "sigma"):
        np.testing.assert_array_equal(np.asarray(a[2][key]), np.asarray(b[2][key]), err_msg=key)
    np.testing.assert_array_equal(a[3], b[3])


@pytest.mark.parametrize("name,storage,n", [("small_gray", "f32", 20), ("qvga_rgb", "f32", 12),
                                            ("qvga_rgb", "bf16", 12), ("vga_rgb", "f32", 6),
                                            ("vga_rgb", "bf16", 6)])
def test_sequence_equals_frame_by_frame(name, storage, n):
    wl = getattr(V, name)()
    frames = _frames(wl, n, storage)
    a = _run(wl, frames, storage, seq=False)
    b = _run(wl, frames, storage, seq=True)
    say(f"{name} {storage} x{n}: launch {b[4]}, fg {int(b[1][2].sum())}")
    _same(a, b)


@pytest.mark.parametrize("mode", [0, 1, 3])
def test_sequence_under_each_exchange(mode):
    wl = V.qvga_rgb()
    frames = _frames(wl, 8, "f32")
    _same(_run(wl, frames, "f32", False, nr=4, mode=mode), _run(wl, frames, "f32", True, nr=4, mode=mode))


def test_sequence_with_rejected_frame_and_reorthonormalization():
    """Frame 3 has a NaN entry (rejected, state unchanged, counted once);
    re-orthonormalisation every 5 frames ends a launch mid-sequence."""
    wl = V.qvga_rgb()
    frames = _frames(wl, 12, "bf16", bad=3)
    a = _run(wl, frames, "bf16", False, reorth_every=5)
    b = _run(wl, frames, "bf16", True, reorth_every=5)
    say(f"status {a[0]} {b[0]}, n {a[1][3]} {b[1][3]}")
    assert a[1][3] == 11
    _same(a, b)


def test_sequence_with_ordinary_dispatch_and_fallback_options():
    wl = V.qvga_rgb()
    frames = _frames(wl, 6, "f32")
    _same(_run(wl, frames, "f32", False), _run(wl, frames, "f32", True, coop=0))
    # filtered-mask weights and pre-processing run one launch per frame
    _same(_run(wl, frames, "f32", False, weights_from_filtered=True),
          _run(wl, frames, "f32", True, weights_from_filtered=True))
    _same(_run(wl, frames, "f32", False, preprocess=True), _run(wl, frames, "f32", True, preprocess=True))


def test_sequence_longer_than_one_launch():
    """300 frames: two launches (256 + 44), still equal to 300 single
    launches."""
    wl = V.small_gray()
    frames = _frames(wl, 300, "f32")
    _same(_run(wl, frames, "f32", False), _run(wl, frames, "f32", True))


def _odd_spec():
    v = V.VideoSpec(41, 29, 3, rank=3, seed=77, noise=0.01, fg_kind="rects", fg_count=2, fg_density=0.1)
    return V.Workload("41x29x3", v, k=6, mu=1e-3, n_frames=20)


@pytest.mark.parametrize("unaligned", [False, True])
def test_bf16_sequence_with_split_pairs_and_unaligned_frames(unaligned):
    """Odd P (row pairs that continue in the next colour plane) and, with
    `unaligned`, frames at an odd bfloat16 offset (no 32-bit pair access):
    the sequence launch still equals one launch per frame."""
    import torch
    wl = _odd_spec()
    frames = _frames(wl, 10, "bf16")
    if unaligned:
        m = frames[0].numel()
        buf = torch.empty(len(frames) * m + 1, dtype=torch.bfloat16, device="cuda")
        views = []
        for i, f in enumerate(frames):
            v = buf[1 + i * m:1 + (i + 1) * m]
            v.copy_(f)
            views.append(v)
        frames = views
    _same(_run(wl, frames, "bf16", False), _run(wl, frames, "bf16", True))
