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
                reorth_every=0, labels_after_update=True, weights_from_filtered=False, preprocess=False,
                ysolve="cg", seed=0):
    """pros_params from keyword arguments (Sec. 5.1 defaults).  seed: the
    draw behind the initial subspace U0 (Sec. 3.4)."""
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
    prm.preprocess = int(bool(preprocess))
    prm.ysolve = {"cg": 0, "gd": 1, "irls": 2}[ysolve]
    prm.seed = int(seed)
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

    def set_preprocess(self, mean=None, m2=None, count=0):
        """Pre-processing statistics (Sec. 3.4): running average, per-entry
        sum of squared deviations (length m each) and the frame count."""
        mv = None if mean is None else np.ascontiguousarray(np.asarray(mean, np.float64))
        vv = None if m2 is None else np.ascontiguousarray(np.asarray(m2, np.float64))
        for v in (mv, vv):
            assert v is None or v.shape == (self.m,)
        L.check(L.lib().pros_set_preprocess(self._h, None if mv is None else _ptr(mv),
                                            None if vv is None else _ptr(vv), int(count)))

    def get_preprocess(self):
        """(mean, m2, count, scale): scale divides the next frame."""
        mv = np.empty(self.m, np.float64)
        vv = np.empty(self.m, np.float64)
        cnt = C.c_int64()
        sc = C.c_double()
        L.check(L.lib().pros_get_preprocess(self._h, _ptr(mv), _ptr(vv), C.byref(cnt), C.byref(sc)))
        return mv, vv, int(cnt.value), float(sc.value)

    def set_score_output(self, scores=None):
        """Have every frame write |r'| of each entry (Step 3 residual) into
        `scores`, a float32 device tensor of m entries (None stops it)."""
        if scores is not None:
            import torch
            assert scores.is_cuda and scores.dtype == torch.float32 and scores.is_contiguous()
            assert scores.numel() == self.m
            self._scores = scores           # keep the buffer alive while registered
        else:
            self._scores = None
        L.check(L.lib().pros_set_score_output(self._h, None if scores is None else _ptr(scores)))

    def quality_counts(self, truth, filtered=True):
        """(TP, FP, TN, FN) of the latest mask (or raw labels) against a
        ground-truth mask of P pixels (host array or device uint8 tensor)."""
        out = np.zeros(4, np.int64)
        if isinstance(truth, np.ndarray):
            t = np.ascontiguousarray(truth.astype(np.uint8).ravel())
            assert t.size == self.P
            L.check(L.lib().pros_quality_counts(self._h, _ptr(t), 0, int(bool(filtered)), _ptr(out)))
        else:
            assert truth.is_cuda and truth.numel() == self.P and truth.is_contiguous()
            L.check(L.lib().pros_quality_counts(self._h, _ptr(truth), 1, int(bool(filtered)), _ptr(out)))
        return tuple(int(v) for v in out)

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

    def track_many(self, frames):
        """Queue a buffered sequence of device tensors (storage dtype, each
        contiguous) through pros_track_frames: the same results as one
        track() per frame, with up to 256 frames per kernel launch."""
        import torch
        frames = list(frames)
        dt = {torch.float32: L.PROS_F32, torch.bfloat16: L.PROS_BF16}[frames[0].dtype]
        for f in frames:
            assert f.is_cuda and f.is_contiguous() and f.numel() == self.m and f.dtype == frames[0].dtype
        ptrs = (C.c_void_p * len(frames))(*[f.data_ptr() for f in frames])
        L.check(L.lib().pros_track_frames(self._h, ptrs, len(frames), dt))

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
                    zeta=s.zeta, nu=s.nu, fg_pixels=s.fg_pixels)

    def sync(self):
        return L.lib().pros_sync(self._h)

    def reorthonormalize(self):
        L.check(L.lib().pros_reorthonormalize(self._h))

    def launch_info(self):
        li = L.pros_launch_info()
        L.check(L.lib().pros_get_launch_info(self._h, C.byref(li)))
        return dict(workgroups=li.workgroups, threads=li.threads, rows_per_thread=li.rows_per_thread,
                    pixels_per_wg=li.pixels_per_wg, barriers_per_frame=li.barriers_per_frame,
                    sync_mode=li.sync_mode, curvature=li.curvature)

    def set_launch(self, rows_per_thread=0, sync_mode=2):
        L.check(L.lib().pros_set_launch(self._h, int(rows_per_thread), int(sync_mode)))

    def set_dispatch(self, cooperative):
        """1: cooperative launches (default); 0: ordinary launches of the
        resident grid (about 17 us less per frame; dedicated device only)."""
        L.check(L.lib().pros_set_dispatch(self._h, int(cooperative)))

    def set_curvature(self, schedule):
        """0: d^T H d in a second pass per CG step; 1: H reduced with the
        gradient (one exchange per step, float32 storage)."""
        L.check(L.lib().pros_set_curvature(self._h, int(schedule)))


def bf16_bits(a):
    """float array -> bfloat16 bit patterns (round to nearest even), uint16."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def bf16_to_f64(b):
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


class BatchTracker:
    """Many independent streams advanced by one persistent launch per step
    (pros_batch_*).  `specs` is a list of dicts with width, height, channels,
    k and any make_params keyword; all streams share one storage type."""

    def __init__(self, specs, storage="f32", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("BatchTracker needs a HIP GPU")
        n = len(specs)
        arr = (L.pros_params * n)()
        self.shapes = []
        for i, sp in enumerate(specs):
            sp = dict(sp)
            w, h, c, k = sp.pop("width"), sp.pop("height"), sp.pop("channels"), sp.pop("k")
            arr[i] = make_params(w, h, c, k, storage=storage, **sp)
            self.shapes.append((w, h, c, k))
        self.n = n
        self.storage = storage
        b = C.c_void_p()
        L.check(L.lib().pros_batch_init(arr, n, _stream_handle(stream), C.byref(b)))
        self._b = b
        self._frames = None

    def close(self):
        if getattr(self, "_b", None):
            L.lib().pros_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _dims(self, s):
        w, h, c, k = self.shapes[s]
        return w * h, w * h * c, k

    def set_state(self, s, U, y=None, labels=None, n=0):
        P, m, k = self._dims(s)
        Ucm = np.ascontiguousarray(np.asarray(U, np.float64).T)
        assert Ucm.shape == (k, m)
        yv = None if y is None else np.ascontiguousarray(np.asarray(y, np.float64))
        lab = None if labels is None else np.ascontiguousarray(np.asarray(labels, np.uint8))
        L.check(L.lib().pros_batch_set_state(self._b, s, _ptr(Ucm), None if yv is None else _ptr(yv),
                                             None if lab is None else _ptr(lab), int(n)))

    def get_preprocess(self, s):
        """Stream s's pre-processing statistics (mean, m2, count, scale)."""
        P, m, k = self._dims(s)
        mv = np.empty(m, np.float64)
        vv = np.empty(m, np.float64)
        cnt = C.c_int64()
        sc = C.c_double()
        L.check(L.lib().pros_batch_get_preprocess(self._b, s, _ptr(mv), _ptr(vv), C.byref(cnt), C.byref(sc)))
        return mv, vv, int(cnt.value), float(sc.value)

    def get_state(self, s):
        P, m, k = self._dims(s)
        Ucm = np.empty((k, m), np.float64)
        y = np.empty(k, np.float64)
        lab = np.empty(P, np.uint8)
        n = C.c_int64()
        L.check(L.lib().pros_batch_get_state(self._b, s, _ptr(Ucm), _ptr(y), _ptr(lab), C.byref(n)))
        return Ucm.T.copy(), y, lab, int(n.value)

    def set_frames(self, frames):
        """frames[s][i]: device tensor of stream s, ring slot i (all streams
        the same ring length).  The tensors are kept alive here."""
        ring = len(frames[0])
        ptrs = (C.c_void_p * (self.n * ring))()
        for s in range(self.n):
            assert len(frames[s]) == ring
            for i, t in enumerate(frames[s]):
                assert t.is_cuda and t.is_contiguous() and t.numel() == self._dims(s)[1]
                ptrs[s * ring + i] = t.data_ptr()
        L.check(L.lib().pros_batch_set_frames(self._b, ptrs, ring))
        self._frames = frames

    def step(self):
        L.check(L.lib().pros_batch_track(self._b))

    def track(self, frames):
        """One batch step on this call's frames: frames[s] is a device tensor
        of stream s (pros_batch_track_frames).  References to the last four
        calls' tensors are kept; synchronise before reusing older ones."""
        assert len(frames) == self.n
        ptrs = (C.c_void_p * self.n)()
        for s, t in enumerate(frames):
            assert t.is_cuda and t.is_contiguous() and t.numel() == self._dims(s)[1]
            ptrs[s] = t.data_ptr()
        L.check(L.lib().pros_batch_track_frames(self._b, ptrs))
        self._recent = (getattr(self, "_recent", []) + [list(frames)])[-4:]

    def steps(self, n):
        """n batch steps in one launch (pros_batch_track_steps)."""
        L.check(L.lib().pros_batch_track_steps(self._b, int(n)))

    def use_graph(self, on=True):
        L.check(L.lib().pros_batch_use_graph(self._b, int(bool(on))))

    def set_dispatch(self, cooperative):
        """1: cooperative launches (default); 0: ordinary launches of the
        resident grid (dedicated device only)."""
        L.check(L.lib().pros_batch_set_dispatch(self._b, int(cooperative)))

    def sync(self):
        return L.lib().pros_batch_sync(self._b)

    def mask(self, s, filtered=True):
        P, _, _ = self._dims(s)
        buf = np.empty(P, np.uint8)
        L.check(L.lib().pros_batch_get_mask(self._b, s, _ptr(buf), int(filtered), 0))
        return buf

    def stats(self, s):
        st = L.pros_stats()
        L.check(L.lib().pros_batch_get_stats(self._b, s, C.byref(st)))
        return dict(frame=st.frame, cg_steps=st.cg_steps, f=list(st.f[:st.cg_steps + 1]), theta=st.theta,
                    updated=st.updated, bad_frame=st.bad_frame)

    def config(self):
        c = L.pros_batch_config()
        L.check(L.lib().pros_batch_get_config(self._b, C.byref(c)))
        return dict(register_budget=c.register_budget, workgroups_per_cu=c.workgroups_per_cu,
                    tile_scale=c.tile_scale, strategy=c.strategy, sync_mode=c.sync_mode,
                    workgroups=c.workgroups, rounds=c.rounds, threads=c.threads)

    def configure(self, register_budget=128, workgroups_per_cu=2, tile_scale=1.0, strategy=0, sync_mode=2,
                  threads=512):
        c = L.pros_batch_config(register_budget, workgroups_per_cu, tile_scale, strategy, sync_mode, 0, 0, threads)
        L.check(L.lib().pros_batch_configure(self._b, C.byref(c)))

    def tune(self, steps=5, cache=None):
        """Pick the fastest launch configuration by timing candidates
        (pros_batch_tune).  With a cache path (or PROST_TUNE_CACHE), a JSON
        file keyed by device, storage and stream shapes remembers the choice."""
        import json
        import os
        import torch
        path = cache or os.environ.get("PROST_TUNE_CACHE")
        key = "|".join([torch.cuda.get_device_properties(0).gcnArchName, self.storage,
                        ";".join("x".join(map(str, s)) for s in self.shapes)])
        if path and os.path.exists(path):
            try:
                db = json.load(open(path))
            except ValueError:
                db = {}
            if key in db:
                self.configure(**db[key]["config"])
                return db[key]
        best = L.pros_batch_config()
        ms = C.c_double()
        L.check(L.lib().pros_batch_tune(self._b, int(steps), C.byref(best), C.byref(ms)))
        rec = dict(config=dict(register_budget=best.register_budget, workgroups_per_cu=best.workgroups_per_cu,
                               tile_scale=best.tile_scale, strategy=best.strategy, sync_mode=best.sync_mode,
                               threads=best.threads),
                   ms_per_step=ms.value, workgroups=best.workgroups, rounds=best.rounds)
        if path:
            db = {}
            if os.path.exists(path):
                try:
                    db = json.load(open(path))
                except ValueError:
                    db = {}
            db[key] = rec
            tmp = path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(db, f, indent=1)
            os.replace(tmp, path)
        return rec


def roc_counts(scores, truth, channels, thresholds, stream=None):
    """Counts (TP, FP, TN, FN) per threshold of the labels
    [max_c scores[c P + p] >= threshold] against truth (device tensors:
    float32 scores of C P entries, uint8 truth of P pixels)."""
    import torch
    assert scores.is_cuda and scores.dtype == torch.float32 and scores.is_contiguous()
    assert truth.is_cuda and truth.dtype == torch.uint8 and truth.is_contiguous()
    P = truth.numel()
    assert scores.numel() == channels * P
    thr = np.ascontiguousarray(np.asarray(thresholds, np.float32))
    out = np.zeros((thr.size, 4), np.int64)
    L.check(L.lib().pros_roc_counts(_ptr(scores), _ptr(truth), int(P), int(channels), _ptr(thr), int(thr.size),
                                    _ptr(out), _stream_handle(stream)))
    return out


def quality_measures(tp, fp, tn, fn):
    """The measures of Sec. 5 from the counts of pros_quality_counts /
    roc_counts: recall, specificity, FPR, FNR, PWC (percent), precision and
    F-measure (nan where a denominator is zero)."""
    nan = float("nan")
    recall = tp / (tp + fn) if tp + fn else nan
    precision = tp / (tp + fp) if tp + fp else nan
    if tp:
        fm = 2.0 * precision * recall / (precision + recall)
    else:
        fm = 0.0 if (fp or fn) else nan
    return {"recall": recall, "specificity": tn / (tn + fp) if tn + fp else nan,
            "fpr": fp / (fp + tn) if fp + tn else nan, "fnr": fn / (tp + fn) if tp + fn else nan,
            "pwc": 100.0 * (fn + fp) / (tp + fn + fp + tn) if tp + fn + fp + tn else nan,
            "precision": precision, "fmeasure": fm}

