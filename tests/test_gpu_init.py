"""The paper's initialization of U (Sec. 3.4) behind the C ABI:
pros_random_subspace against the oracle's draw (Philox4x32-10 + Box-Muller,
reduced QR with diag(R) > 0) entry by entry, U0 of pros_init /
pros_batch_init against the oracle's U0 rounded to the storage type, and a
tracker started from it (no pros_set_state) against the oracle started from
the same U0."""
import ctypes as C

import numpy as np
import pytest

from gpu_common import oracle_params, say, tracker_kwargs
from oracle import prost_oracle as O
from synth import video as V

pytestmark = pytest.mark.gpu


def _device_subspace(seed, stream, m, k):
    import torch
    from paper_1302_2073_amd import _lib as L
    t = torch.full((k, m), float("nan"), dtype=torch.float64, device="cuda")   # column-major m x k
    L.check(L.lib().pros_random_subspace(seed, stream, m, k, C.c_void_p(t.data_ptr()),
                                         C.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return t.cpu().numpy().T.copy()


@pytest.mark.parametrize("m,k,seed,stream", [(4800, 5, 1, 0), (921600, 15, 3, 0), (777, 16, 12345678901, 7),
                                             (16, 16, 0, 0), (4801, 3, 2, 1)])
def test_random_subspace_matches_oracle(m, k, seed, stream):
    say(f"random subspace m={m} k={k} seed={seed} stream={stream}")
    U = _device_subspace(seed, stream, m, k)
    E = O.initial_subspace(m, k, seed, stream)
    err = float(np.max(np.abs(U - E)))
    orth = O.orthonormality_error(U)
    say(f"  max |U - U_oracle| = {err:.2e}, ||U^T U - I||_F = {orth:.2e}")
    assert err <= 1e-12
    assert orth <= 1e-12
    assert np.array_equal(U, _device_subspace(seed, stream, m, k))        # reproducible bit for bit
    assert np.max(np.abs(U - _device_subspace(seed, stream + 1, m, k))) > 1e-3   # distinct per stream


def test_random_subspace_argument_errors():
    import torch
    from paper_1302_2073_amd import _lib as L
    lib = L.lib()
    t = torch.zeros(8, dtype=torch.float64, device="cuda")
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.pros_random_subspace(1, 0, 4, 5, C.c_void_p(t.data_ptr()), s) == L.PROS_EINVAL    # k > m
    assert lib.pros_random_subspace(1, 0, 4, 17, C.c_void_p(t.data_ptr()), s) == L.PROS_EINVAL   # k > 16
    assert lib.pros_random_subspace(1, 0, 4, 2, None, s) == L.PROS_EINVAL


def _ulp32(x):
    return np.spacing(np.abs(x).astype(np.float32)).astype(np.float64)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_init_starts_from_the_seeded_subspace(storage):
    from paper_1302_2073_amd import Tracker
    from paper_1302_2073_amd.tracker import bf16_bits
    w, h, c, k, seed = 160, 120, 3, 10, 77
    with Tracker(w, h, c, k, storage=storage, seed=seed) as trk:
        U, y, lab, n = trk.get_state()
    E = O.initial_subspace(w * h * c, k, seed, 0)
    if storage == "f32":
        ref = E.astype(np.float32).astype(np.float64)
        tol = _ulp32(E)                       # the device's float64 value may round the other way at a tie
    else:
        ref = (bf16_bits(E).astype(np.uint32) << 16).view(np.float32).astype(np.float64)
        tol = 2.0 ** -7 * np.abs(ref)         # one bfloat16 ulp
    err = np.abs(U - ref)
    say(f"  {storage}: entries off the rounded oracle U0: {int(np.sum(err > 0))}, worst {float(np.max(err / np.maximum(tol, 1e-300))):.2f} ulp")
    assert np.all(err <= tol)
    assert np.all(y == 0) and np.all(lab == 0) and n == 0


def test_batch_streams_start_from_distinct_subspaces():
    from paper_1302_2073_amd.tracker import BatchTracker
    specs = [dict(width=80, height=60, channels=1, k=5, seed=5), dict(width=80, height=60, channels=1, k=5, seed=5),
             dict(width=40, height=30, channels=3, k=4, seed=9)]
    bt = BatchTracker(specs, storage="f32")
    try:
        for s, sp in enumerate(specs):
            U = bt.get_state(s)[0]
            E = O.initial_subspace(sp["width"] * sp["height"] * sp["channels"], sp["k"], sp["seed"], s)
            assert np.all(np.abs(U - E.astype(np.float32)) <= _ulp32(E)), s
        assert np.max(np.abs(bt.get_state(0)[0] - bt.get_state(1)[0])) > 1e-3
    finally:
        bt.close()


def test_tracker_from_seeded_u0_follows_the_oracle():
    """200 frames of the 80x60 workload from pros_init's own U0 (no state
    injection) beside the oracle started from its U0 of the same seed:
    label disagreement at most 0.5% of pixels in every frame."""
    from paper_1302_2073_amd import Tracker
    wl = V.small_gray()
    v = wl.video
    prm = oracle_params(wl)
    seed = 31
    st = O.initial_state(O.initial_subspace(prm.m, prm.k, seed, 0), prm.P)
    sv = V.SyntheticVideo(v)
    worst, worst_ang = 0.0, 0.0
    with Tracker(v.width, v.height, v.channels, wl.k, seed=seed, **tracker_kwargs(prm)) as trk:
        for n in range(200):
            x = sv.frame(n).astype(np.float32)
            st, _ = O.track_frame(st, x.astype(np.float64), prm)
            trk.track(x)
            U, y, lab, nn = trk.get_state()
            dis = float(np.mean(lab != st.labels))
            ang = float(O.principal_angles(st.U, U).max())
            worst, worst_ang = max(worst, dis), max(worst_ang, ang)
            if n % 40 == 39:
                say(f"  frame {n}: angle {ang:.2e} y_rel {np.linalg.norm(y - st.y) / np.linalg.norm(st.y):.2e} "
                    f"label disagreement {dis:.4%}")
    say(f"  worst label disagreement {worst:.4%}, worst principal angle {worst_ang:.2e}")
    assert worst <= 0.005
