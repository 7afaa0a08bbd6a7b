"""GPU parity of the segmentation-quality path (Sec. 5 measures and the
delta sweep): per-entry label scores written by the frame kernel, counts of
the mask against planted ground truth, and ROC counts over thresholds."""
import numpy as np
import pytest

from gpu_common import f32, oracle_trajectory, say, tracker_kwargs
from oracle import prost_oracle as O
from synth import video as V

pytestmark = pytest.mark.gpu


def _tracker(prm, storage="f32"):
    from paper_1302_2073_amd import Tracker
    return Tracker(prm.width, prm.height, prm.channels, prm.k, **tracker_kwargs(prm, storage))


@pytest.mark.parametrize("name,frame,storage", [("small_gray", 30, "f32"), ("qvga_rgb", 6, "f32"),
                                                ("qvga_rgb", 6, "bf16")])
def test_scores_match_labels_and_oracle(name, frame, storage):
    """The labels are exactly [max_c score >= delta] of the written scores,
    and the scores match the oracle's Step 3 residual of the same frame."""
    import torch
    from paper_1302_2073_amd.tracker import bf16_bits
    wl, prm, sv, states = oracle_trajectory(name, frame)
    st = states[frame]
    x64 = f32(sv.frame(frame))
    with _tracker(prm, storage) as trk:
        sc = torch.zeros(prm.m, dtype=torch.float32, device="cuda")
        trk.set_score_output(sc)
        trk.set_state(st.U, st.y, st.labels, st.n)
        U0, y0, l0, n0 = trk.get_state()
        if storage == "bf16":
            bits = bf16_bits(x64)
            x64 = bits.astype(np.uint32).__lshift__(16).view(np.float32).astype(np.float64)
            trk.track(bits)
        else:
            trk.track(x64.astype(np.float32))
        U1, y1, l1, n1 = trk.get_state()
        scores = sc.cpu().numpy().astype(np.float64)
        trk.set_score_output(None)
    s_pix = scores.reshape(prm.channels, -1).max(axis=0)
    assert np.array_equal(l1, (s_pix >= np.float32(prm.thr)).astype(np.uint8))
    start = O.State(U0, y0, l0, O.median3x3(l0, prm.height, prm.width), n0)
    exp, _ = O.track_frame(start, x64, prm)
    ref = np.abs(x64 - exp.U @ exp.y)
    err = np.abs(scores - ref)
    say(f"  {name} {storage}: max |score - oracle| {err.max():.2e}")
    assert np.all(err <= 1e-5 + 1e-4 * np.abs(ref))


def test_quality_counts_against_planted_truth():
    """60 frames of the 80x60 workload: the device counts of the mask and of
    the raw labels against the planted mask equal the counts of the same
    masks computed on the host, and the tracker separates the objects."""
    wl, prm, sv, states = oracle_trajectory("small_gray", 0)
    with _tracker(prm) as trk:
        trk.set_state(states[0].U, states[0].y, states[0].labels, 0)
        for n in range(60):
            x, truth = sv.frame(n, with_mask=True)
            trk.track(x.astype(np.float32))
        for filtered in (True, False):
            got = trk.quality_counts(truth, filtered)
            mask = trk.mask(filtered=filtered)
            assert got == O.quality_counts(mask, truth)
        q = O.quality_metrics(*trk.quality_counts(truth, True))
    say(f"  frame 59 quality: {q}")
    assert q["recall"] > 0.5 and q["specificity"] > 0.9


def test_roc_counts_match_host_sweep():
    import torch
    from paper_1302_2073_amd import roc_counts
    wl, prm, sv, states = oracle_trajectory("qvga_rgb", 0)
    with _tracker(prm) as trk:
        sc = torch.zeros(prm.m, dtype=torch.float32, device="cuda")
        trk.set_score_output(sc)
        trk.set_state(states[0].U, states[0].y, states[0].labels, 0)
        for n in range(20):
            x, truth = sv.frame(n, with_mask=True)
            trk.track(x.astype(np.float32))
        trk.sync()
        thr = np.linspace(0.02, 0.6, 30).astype(np.float32)
        tdev = torch.from_numpy(truth.astype(np.uint8)).cuda()
        got = roc_counts(sc, tdev, prm.channels, thr)
        s_pix = sc.cpu().numpy().astype(np.float64).reshape(prm.channels, -1).max(axis=0)
        trk.set_score_output(None)
    ref = np.array(O.roc_counts(s_pix, truth, thr.astype(np.float64)))
    assert np.array_equal(got, ref)
    pts = [(fp / (fp + tn), tp / (tp + fn)) for tp, fp, tn, fn in got]
    say(f"  ROC (FPR, recall) at delta = {thr[0]:.2f} .. {thr[-1]:.2f}: {pts[0]} .. {pts[-1]}")
    assert all(a[0] >= b[0] and a[1] >= b[1] for a, b in zip(pts, pts[1:]))   # monotone in delta

