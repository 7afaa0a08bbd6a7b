"""Video ingest around a tracker (argument marshalling only; the work runs in
libprost.so): area re-sampling of interleaved 8-bit frames to the tracker's
resolution (Sec. 5.1 tracks every sequence at 160 x 120), nearest-neighbour
upsampling of the mask back to the source size (Sec. 5.3), and a pinned,
double-buffered host-to-device pipeline."""
import ctypes as C

import numpy as np

from . import _lib as L
from .tracker import _ptr, _stream_handle

_DTYPES = {"f32": L.PROS_F32, "bf16": L.PROS_BF16}


def resample_rgb8(src, dst_w, dst_h, dtype="f32", scale=1.0 / 255.0, out=None, stream=None):
    """src: uint8 device tensor H x W x C (rows may be padded: a strided
    view of the last two dimensions contiguous).  Returns the planar frame
    (C * dst_h * dst_w entries, float32 or bfloat16) of area averages times
    `scale`."""
    import torch
    assert src.is_cuda and src.dtype == torch.uint8 and src.dim() in (2, 3)
    img = src if src.dim() == 3 else src.unsqueeze(2)
    H, W, Cc = img.shape
    assert (Cc == 1 or img.stride(2) == 1) and (W == 1 or img.stride(1) == Cc), "pixels must be packed within a row"
    row_stride = img.stride(0) if H > 1 else W * Cc
    tdt = torch.float32 if dtype == "f32" else torch.bfloat16
    if out is None:
        out = torch.empty(Cc * dst_h * dst_w, dtype=tdt, device=src.device)
    assert out.is_cuda and out.dtype == tdt and out.is_contiguous() and out.numel() == Cc * dst_h * dst_w
    L.check(L.lib().pros_resample_rgb8(_ptr(img), int(W), int(H), int(Cc), int(row_stride), _ptr(out),
                                       _DTYPES[dtype], int(dst_w), int(dst_h), float(scale), _stream_handle(stream)))
    return out


def mask_upsample(mask, width, height, out_w, out_h, stream=None):
    """mask: uint8 device tensor of height * width labels -> out_h * out_w
    labels by nearest neighbour (pixel centres)."""
    import torch
    assert mask.is_cuda and mask.dtype == torch.uint8 and mask.is_contiguous() and mask.numel() == width * height
    out = torch.empty(out_w * out_h, dtype=torch.uint8, device=mask.device)
    L.check(L.lib().pros_mask_upsample(_ptr(mask), int(width), int(height), _ptr(out), int(out_w), int(out_h),
                                       _stream_handle(stream)))
    return out


class Ingest:
    """pros_ingest_*: host frames (src_h x src_w x C uint8) -> pinned slot ->
    copy stream -> resample + track on the tracker's stream."""

    def __init__(self, tracker, src_w, src_h, slots=2, scale=1.0 / 255.0):
        self.tracker = tracker
        self.src_w, self.src_h = int(src_w), int(src_h)
        self.channels = int(tracker.params.channels)
        self.nbytes = self.src_w * self.src_h * self.channels
        g = C.c_void_p()
        L.check(L.lib().pros_ingest_init(tracker._h, self.src_w, self.src_h, int(slots), float(scale), C.byref(g)))
        self._g = g

    def close(self):
        if self._g is not None:
            L.lib().pros_ingest_destroy(self._g)
            self._g = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def slot(self):
        """The next pinned host buffer as a writable (H, W, C) uint8 array."""
        p = C.c_void_p()
        L.check(L.lib().pros_ingest_slot(self._g, C.byref(p)))
        buf = (C.c_uint8 * self.nbytes).from_address(p.value)
        return np.frombuffer(buf, dtype=np.uint8).reshape(self.src_h, self.src_w, self.channels)

    def submit(self):
        L.check(L.lib().pros_ingest_submit(self._g))

    def push(self, frame):
        """Copy one host frame (H x W x C uint8) through the pipeline."""
        f = np.ascontiguousarray(frame, dtype=np.uint8)
        assert f.size == self.nbytes
        L.check(L.lib().pros_ingest_push(self._g, _ptr(f)))

    def mask(self, filtered=True, out=None):
        """Latest mask upsampled to the source size: into a uint8 device tensor
        `out` (queued), else returned as a host array (synchronises)."""
        if out is not None:
            assert out.is_cuda and out.numel() == self.src_w * self.src_h
            L.check(L.lib().pros_ingest_mask(self._g, _ptr(out), int(bool(filtered)), 1))
            return out
        host = np.empty(self.src_w * self.src_h, np.uint8)
        L.check(L.lib().pros_ingest_mask(self._g, _ptr(host), int(bool(filtered)), 0), allow=(L.PROS_EBADFRAME,))
        return host
