"""Host check of the wavefront lane-exchange schedule used by every kernel's
reductions (the reduce-scatter and the 16-lane / 64-lane sums): the stage
order and DPP controls are read from the device header and replayed on a
64-lane model of the gfx950 primitives, whose lane semantics were checked
on the device (permlane swaps, row rotations: lane l reads lane l - r mod 16
of its row, quad permutations).  Each component must end in exactly one
owner lane with the wavefront total, and every lane of a 16-lane row must
hold the same row total."""
import os
import re

import numpy as np
import pytest

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_1302_2073_amd", "csrc", "prost_device.hpp")


def _consts():
    src = open(HDR).read()
    order = [int(x) for x in re.search(r"kRsOrder\[6\]\s*=\s*\{([^}]*)\}", src).group(1).split(",")]
    c = {}
    for name in ("kRowRor4", "kRowRor8", "kRowRor12", "kQuadXor1", "kQuadXor2"):
        c[name] = int(re.search(name + r"\s*=\s*(0x[0-9A-Fa-f]+)", src).group(1), 16)
    return order, c


ORDER, CTRL = _consts()
LANES = np.arange(64)


def dpp(v, ctrl):
    if 0x121 <= ctrl <= 0x12F:                       # row_ror:r
        r = ctrl - 0x120
        return v[(LANES & ~15) + ((LANES - r) % 16)]
    if ctrl <= 0xFF:                                 # quad_perm
        p = [(ctrl >> (2 * i)) & 3 for i in range(4)]
        return v[(LANES & ~3) + np.array(p)[LANES & 3]]
    raise ValueError(hex(ctrl))


def permlane_swap(x, y, w):
    xs, ys = x.copy(), y.copy()
    upper = ((LANES // w) & 1) == 1                  # odd blocks of w lanes within each 2w
    xs[upper] = y[LANES[upper] - w]
    ys[~upper] = x[LANES[~upper] + w]
    return xs, ys


def rs_stage(b, lo, hi):
    if b in (5, 4):
        x, y = permlane_swap(lo, hi, 32 if b == 5 else 16)
        return x + y
    up = ((LANES >> b) & 1) == 1
    send, keep = np.where(up, lo, hi), np.where(up, hi, lo)
    ctrl = {3: CTRL["kRowRor8"], 0: CTRL["kQuadXor1"], 1: CTRL["kQuadXor2"]}[b]
    return keep + dpp(send, ctrl)


def ar_stage(b, v):
    if b in (5, 4):
        x, y = permlane_swap(v, v, 32 if b == 5 else 16)
        return x + y
    ctrl = {3: CTRL["kRowRor8"], 0: CTRL["kQuadXor1"], 1: CTRL["kQuadXor2"], 2: CTRL["kRowRor12"]}[b]
    return v + dpp(v, ctrl)


def reduce_scatter(a):
    L = a.shape[0]
    P = 1 << max(L - 1, 0).bit_length()
    S = P.bit_length() - 1
    a = [a[i].copy() for i in range(L)] + [np.zeros(64, a.dtype)] * (P - L)
    base = np.zeros(64, int)
    for st in range(S):
        half = P >> (st + 1)
        b = ORDER[st]
        a = [rs_stage(b, a[i], a[i + half]) for i in range(half)]
        base += np.where((LANES >> b) & 1, half, 0)
    v = a[0]
    for st in range(S, 6):
        v = ar_stage(ORDER[st], v)
    owner_mask = sum(1 << ORDER[st] for st in range(S, 6))
    return v, base, (LANES & owner_mask) == 0


@pytest.mark.parametrize("L", [1, 2, 3, 5, 8, 11, 16, 17, 32])
def test_reduce_scatter_owners_hold_each_total_once(L):
    rng = np.random.default_rng(L)
    a = rng.integers(-1000, 1000, size=(L, 64)).astype(np.int64)   # integers: sums are exact
    v, comp, owner = reduce_scatter(a)
    want = a.sum(axis=1)
    got = {}
    for lane in np.flatnonzero(owner):
        c = int(comp[lane])
        if c < L:
            assert c not in got, f"component {c} owned twice"
            got[c] = int(v[lane])
    assert sorted(got) == list(range(L))
    assert all(got[c] == want[c] for c in range(L))


def test_row_and_wave_sums():
    rng = np.random.default_rng(7)
    v = rng.standard_normal(64).astype(np.float32)
    r = v.copy()
    for ctrl in (CTRL["kRowRor8"], CTRL["kRowRor4"], CTRL["kQuadXor2"], CTRL["kQuadXor1"]):
        r = r + dpp(r, ctrl)
    rows = r.reshape(4, 16)
    assert (rows == rows[:, :1]).all()                                  # one total per row, bit-identical
    assert np.allclose(rows[:, 0], v.reshape(4, 16).sum(axis=1), rtol=1e-5)
    w = v.copy()
    for width in (32, 16):
        x, y = permlane_swap(w, w, width)
        w = x + y
    for ctrl in (CTRL["kRowRor8"], CTRL["kRowRor4"], CTRL["kQuadXor2"], CTRL["kQuadXor1"]):
        w = w + dpp(w, ctrl)
    assert (w == w[0]).all() and np.isclose(w[0], v.sum(), rtol=1e-5)
