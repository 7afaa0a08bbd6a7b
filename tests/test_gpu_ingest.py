"""GPU parity of the ingest path: area re-sampling of interleaved 8-bit
frames to the tracker's resolution (Sec. 5.1), nearest-neighbour upsampling
of the mask (Sec. 5.3), and the pinned pipeline, which must give exactly the
state of resample + track issued by hand."""
import numpy as np
import pytest

from gpu_common import say
from oracle import prost_oracle as O
from synth import video as V

pytestmark = pytest.mark.gpu

SIZES = [((640, 480), (160, 120)), ((352, 288), (160, 120)), ((123, 77), (160, 120)), ((1920, 1080), (160, 120)),
         ((160, 120), (160, 120)), ((1, 1), (5, 3)), ((37, 29), (1, 1)), ((1023, 7), (64, 5))]


def _bf16_ulp(v):
    m, e = np.frexp(np.abs(v))           # v = m 2^e, m in [0.5, 1)
    return np.ldexp(1.0, e - 8)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("src,dst", SIZES)
def test_resample_matches_oracle(src, dst, dtype):
    """Every entry is the area mean rounded once: within one unit in the last
    place of the output type of the float64 oracle."""
    import torch
    from paper_1302_2073_amd.ingest import resample_rgb8
    (W, H), (w, h) = src, dst
    img = V.CameraVideo(W, H, 3, seed=W + H).frame(3)
    say(f"resample {W}x{H} -> {w}x{h} {dtype}")
    ref = O.resample_area(img, w, h)
    out = resample_rgb8(torch.from_numpy(img).cuda(), w, h, dtype)
    torch.cuda.synchronize()
    got = out.float().cpu().numpy().astype(np.float64)
    assert got.shape == ref.shape
    if dtype == "f32":
        tol = np.spacing(ref.astype(np.float32)).astype(np.float64)
    else:
        tol = _bf16_ulp(ref)
    bad = np.abs(got - ref) > tol
    assert not bad.any(), (int(bad.sum()), float(np.abs(got - ref).max()))


def test_resample_padded_rows_and_gray():
    """Rows with padding bytes (a decoder's pitch) and one channel."""
    import torch
    from paper_1302_2073_amd.ingest import resample_rgb8
    img = V.CameraVideo(100, 60, 1, seed=7).frame(2)
    pad = np.zeros((60, 128, 1), np.uint8)
    pad[:, :100] = img
    dev = torch.from_numpy(pad).cuda()[:, :100]          # row stride 128 bytes
    out = resample_rgb8(dev, 40, 24, "f32", scale=1.0)
    torch.cuda.synchronize()
    ref = O.resample_area(img, 40, 24, scale=1.0)
    np.testing.assert_array_less(np.abs(out.cpu().numpy() - ref), np.spacing(ref.astype(np.float32)) + 1e-30)


@pytest.mark.parametrize("src,dst", [((160, 120), (640, 480)), ((160, 120), (352, 288)), ((7, 5), (16, 9)),
                                     ((5, 3), (1, 1)), ((33, 17), (33, 17)), ((64, 48), (20, 15))])
def test_mask_upsample_bit_exact(src, dst):
    import torch
    from paper_1302_2073_amd.ingest import mask_upsample
    (w, h), (ow, oh) = src, dst
    m = (np.random.default_rng(w * h).random(w * h) < 0.3).astype(np.uint8)
    out = mask_upsample(torch.from_numpy(m).cuda(), w, h, ow, oh)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), O.mask_upsample(m, w, h, ow, oh))


@pytest.mark.parametrize("storage,slots", [("f32", 2), ("f32", 1), ("bf16", 3)])
def test_pipeline_equals_resample_then_track(storage, slots):
    """640x480 camera frames through the pinned pipeline (push and
    slot/submit alternately) against the same frames resampled to 160x120 and
    tracked by hand: identical state, labels and upsampled mask."""
    import torch
    from paper_1302_2073_amd import Tracker
    from paper_1302_2073_amd.ingest import Ingest, resample_rgb8
    cam = V.CameraVideo(640, 480, 3, seed=21)
    w, h, k = 160, 120, 15
    kw = dict(mu=1e-3, storage=storage, i_init=20)
    U0 = V.initial_subspace(w * h * 3, k, 9)
    with Tracker(w, h, 3, k, **kw) as a, Tracker(w, h, 3, k, **kw) as b:
        a.set_state(U0)
        b.set_state(U0)
        with Ingest(a, 640, 480, slots=slots) as ing:
            for n in range(8):
                f = cam.frame(n)
                if n % 2:
                    ing.push(f)
                else:
                    ing.slot()[...] = f
                    ing.submit()
                b.track(resample_rgb8(torch.from_numpy(f).cuda(), w, h, storage))
            up = ing.mask(filtered=True)
            up_dev = ing.mask(filtered=False, out=torch.empty(640 * 480, dtype=torch.uint8, device="cuda"))
            torch.cuda.synchronize()
            Ua, ya, la, na = a.get_state()
            Ub, yb, lb, nb = b.get_state()
            say(f"pipeline {storage} slots={slots}: n={na} fg={int(la.sum())}")
            assert na == nb == 8
            np.testing.assert_array_equal(Ua, Ub)
            np.testing.assert_array_equal(ya, yb)
            np.testing.assert_array_equal(la, lb)
            np.testing.assert_array_equal(up, O.mask_upsample(b.mask(filtered=True), w, h, 640, 480))
            np.testing.assert_array_equal(up_dev.cpu().numpy(), O.mask_upsample(lb, w, h, 640, 480))


def test_pipeline_refusals():
    from paper_1302_2073_amd import Tracker
    from paper_1302_2073_amd._lib import ProstError
    from paper_1302_2073_amd.ingest import Ingest
    with Tracker(16, 12, 3, 2) as t:
        with pytest.raises(ProstError):
            Ingest(t, 0, 10)
        with pytest.raises(ProstError):
            Ingest(t, 32, 24, slots=0)
        with Ingest(t, 32, 24) as ing:
            with pytest.raises(ProstError):     # no slot filled yet
                ing.submit()
            ing.push(np.zeros((24, 32, 3), np.uint8))   # tracks from the seeded U0 of pros_init (Sec. 3.4)
            assert t.get_state()[3] == 1
