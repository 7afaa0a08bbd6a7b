"""Python front end of the pROST C ABI: one video stream per Tracker.

Argument marshalling only.  Every step of the frame runs in the HIP kernels
of libprost.so; torch supplies device memory and the HIP stream.
"""
from __future__ import annotations

import ctypes as C
import math
from typing import Optional

import numpy as np

from . import _lib as L


def make_params(width, height, channels=1, k=15, cg_iters=5, cost="lp", p=0.25, mu=1e-3,
                delta=None, omega=5e-5, t_init=5e-3, t_min=1e-4, i_init=100, storage="f32",
                reorth_every=0, labels_after_update=True, weights_from_filtered=False):
    """pros_params from keyword arguments (Sec. 5.1 defaults)."""
    prm = L.pros_params()
    L.check(L.lib().pros_params_default(C.byref(prm), width, height, channels))
    prm.k = k
    prm.cg_iters = cg_iters
    prm.cost = {"lp": L.PROS_COST_LP, "log": L.PROS_COST_LOG}[cost]
    prm.p = p
    prm.mu = mu
    prm.delta = 0.0 if delta is None else float(delta)
    prm.omega = omega
    prm.t_init = t_init
    prm.t_min = t_min
    prm.i_init = int(i_init)
    prm.storage = {"f32": L.PROS_F32, "bf16": L.PROS_BF16}[storage]
    prm.reorth_every = int(reorth_every)
    prm.labels_after_update = int(bool(labels_after_update))
    prm.weights_from_filtered = int(bool(weights_from_filtered))
    return prm


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(a):
    """Data pointer of a numpy array or a torch tensor."""
    if isinstance(a, np.ndarray):
        return C.c_void_p(a.ctypes.data)
    return C.c_void_p(a.data_ptr())


class Tracker:
    """pros_init / pros_track_frame / pros_get_mask for one stream."""

    def __init__(self, width, height, channels=1, k=15, stream=None, **kw):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Tracker needs a HIP GPU")
        self.params = make_params(width, height, channels, k, **kw)
        self.width, self.height, self.channels, self.k = width, height, channels, k
        self.P = width * height
        self.m = self.P * channels
        self.storage = kw.get("storage", "f32")
        self._stream = stream
        h = C.c_void_p()
        L.check(L.lib().pros_init(C.byref(self.params), _stream_handle(stream), C.byref(h)))
        self._h = h

    # -- lifetime --------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            L.lib().pros_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- state -----------------------------------------------------------
    def set_state(self, U, y=None, labels=None, n=0):
        U = np.asarray(U, dtype=np.float64)
        assert U.shape == (self.m, self.k), U.shape
        Ucm = np.ascontiguousarray(U.T)           # column-major m x k
        yv = None if y is None else np.ascontiguousarray(np.asarray(y, dtype=np.float64))
        lab = None if labels is None else np.ascontiguousarray(np.asarray(labels, dtype=np.uint8))
        L.check(L.lib().pros_set_state(self._h, _ptr(Ucm), None if yv is None else _ptr(yv),
                                       None if lab is None else _ptr(lab), int(n)))

    def get_state(self):
        Ucm = np.empty((self.k, self.m), np.float64)
        y = np.empty(self.k, np.float64)
        lab = np.empty(self.P, np.uint8)
        n = C.c_int64()
        L.check(L.lib().pros_get_state(self._h, _ptr(Ucm), _ptr(y), _ptr(lab), C.byref(n)))
        return Ucm.T.copy(), y, lab, int(n.value)

    # -- frames ----------------------------------------------------------
    def track(self, frame):
        """Queue one frame: a device tensor of the storage dtype (read in
        place) or a host array (float32 or bfloat16-as-uint16)."""
        if isinstance(frame, np.ndarray):
            if frame.dtype == np.float32:
                dt = L.PROS_F32
            elif frame.dtype == np.uint16:
                dt = L.PROS_BF16
            else:
                raise TypeError("host frames are float32 or bfloat16 bits (uint16)")
            frame = np.ascontiguousarray(frame)
            st = L.lib().pros_track_frame(self._h, _ptr(frame), dt, 0)
        else:
            import torch
            dt = {torch.float32: L.PROS_F32, torch.bfloat16: L.PROS_BF16}[frame.dtype]
            assert frame.is_cuda and frame.is_contiguous() and frame.numel() == self.m
            st = L.lib().pros_track_frame(self._h, _ptr(frame), dt, 1)
        L.check(st)

    def mask(self, filtered=True, out=None):
        if out is not None:       # device tensor of P uint8, queued on the stream
            L.check(L.lib().pros_get_mask(self._h, _ptr(out), int(filtered), 1))
            return out
        buf = np.empty(self.P, np.uint8)
        L.check(L.lib().pros_get_mask(self._h, _ptr(buf), int(filtered), 0))
        return buf

    def stats(self):
        s = L.pros_stats()
        L.check(L.lib().pros_get_stats(self._h, C.byref(s)))
        steps = s.cg_steps
        return dict(frame=s.frame, cg_steps=steps, restarts=s.restarts, updated=s.updated,
                    bad_frame=s.bad_frame, f=list(s.f[:steps + 1]), alpha=list(s.alpha[:steps]),
                    beta=list(s.beta[:steps]), t=s.t, sigma=s.sigma, theta=s.theta,
                    zeta=s.zeta, nu=s.nu)

    def sync(self):
        return L.lib().pros_sync(self._h)

    def reorthonormalize(self):
        L.check(L.lib().pros_reorthonormalize(self._h))

    def launch_info(self):
        li = L.pros_launch_info()
        L.check(L.lib().pros_get_launch_info(self._h, C.byref(li)))
        return dict(workgroups=li.workgroups, threads=li.threads, rows_per_thread=li.rows_per_thread,
                    pixels_per_wg=li.pixels_per_wg, barriers_per_frame=li.barriers_per_frame)


def bf16_bits(a):
    """float array -> bfloat16 bit patterns (round to nearest even), uint16."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def bf16_to_f64(b):
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)
