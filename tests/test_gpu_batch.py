"""GPU parity of the batched form: uneven streams advanced by one persistent
launch per step, each stream against its own float64 oracle run."""
import numpy as np
import pytest

from gpu_common import GUARD, TOL_U, TOL_Y, f32, say, update_rounding_bound
from oracle import prost_oracle as O
from synth import video as V

pytestmark = pytest.mark.gpu

SHAPES = [(80, 60, 1, 5), (64, 48, 3, 10), (160, 120, 3, 15), (37, 23, 3, 16), (33, 17, 2, 1)]


def _streams(shapes=SHAPES, warm=4):
    out = []
    for i, (W, H, Cc, k) in enumerate(shapes):
        spec = V.VideoSpec(W, H, Cc, rank=min(k, 3), seed=40, stream=i, noise=0.01, fg_kind="rects",
                           fg_count=2, fg_density=0.08)
        sv = V.SyntheticVideo(spec)
        prm = O.Params(W, H, Cc, k=k, mu=1e-3, i_init=20)
        st = O.initial_state(V.initial_subspace(prm.m, k, 40, i), prm.P)
        for n in range(warm):
            st, _ = O.track_frame(st, f32(sv.frame(n)), prm)
        out.append((sv, prm, st))
    return out


def _specs(streams):
    return [dict(width=p.width, height=p.height, channels=p.channels, k=p.k, mu=p.mu, i_init=p.i_init)
            for _, p, _ in streams]


def _frames_tensor(streams, n0, ring, dtype="f32"):
    import torch
    from paper_1302_2073_amd.tracker import bf16_bits
    fr = []
    for sv, prm, _ in streams:
        row = []
        for i in range(ring):
            x = sv.frame(n0 + i)
            if dtype == "f32":
                row.append(torch.from_numpy(x.astype(np.float32)).cuda())
            else:
                row.append(torch.from_numpy(bf16_bits(x).view(np.int16)).cuda().view(torch.bfloat16))
        fr.append(row)
    return fr


def _check_stream(bt, s, prm, start_state, x64):
    exp, info = O.track_frame(start_state, x64, prm)
    U1, y1, l1, n1 = bt.get_state(s)
    band = O.band_pixels(exp.U, x64, exp.y, prm.thr, prm.channels, GUARD)
    y_rel = np.linalg.norm(y1 - exp.y) / np.linalg.norm(exp.y)
    U_rel = np.linalg.norm(U1 - exp.U) / np.linalg.norm(exp.U)
    mism = int(np.sum((l1 != exp.labels) & ~band))
    mask = bt.mask(s)
    say(f"  stream {s} {prm.width}x{prm.height}x{prm.channels} k={prm.k}: y {y_rel:.1e} U {U_rel:.1e} "
        f"labels outside band {mism} (band {int(band.sum())})")
    assert n1 == exp.n
    assert y_rel <= TOL_Y and U_rel <= TOL_U and mism == 0
    assert np.array_equal(mask, O.median3x3(l1, prm.height, prm.width))
    return exp


def _load(bt, streams):
    starts = []
    for s, (sv, prm, st) in enumerate(streams):
        bt.set_state(s, st.U, st.y, st.labels, st.n)
        U0, y0, l0, n0 = bt.get_state(s)
        starts.append(O.State(U0, y0, l0, O.median3x3(l0, prm.height, prm.width), n0))
    return starts


@pytest.mark.parametrize("cfg", [dict(register_budget=128, workgroups_per_cu=2, tile_scale=1.0, strategy=0),
                                 dict(register_budget=64, workgroups_per_cu=1, tile_scale=0.5, strategy=1),
                                 dict(register_budget=128, workgroups_per_cu=1, tile_scale=1.0, strategy=0,
                                      sync_mode=0),
                                 dict(register_budget=128, workgroups_per_cu=1, tile_scale=0.75, strategy=0,
                                      sync_mode=2)])
def test_batch_step_matches_oracle_per_stream(cfg):
    from paper_1302_2073_amd.tracker import BatchTracker
    streams = _streams()
    with BatchTracker(_specs(streams)) as bt:
        bt.configure(**cfg)
        say("  config", bt.config())
        fr = _frames_tensor(streams, 4, 2)
        bt.set_frames(fr)
        starts = _load(bt, streams)
        bt.step()
        assert bt.sync() == 0
        nxt = []
        for s, (sv, prm, st) in enumerate(streams):
            nxt.append(_check_stream(bt, s, prm, starts[s], f32(sv.frame(4))))
        # second step reads ring slot 1, continuing from the GPU's own state
        starts2 = []
        for s, (sv, prm, st) in enumerate(streams):
            U0, y0, l0, n0 = bt.get_state(s)
            starts2.append(O.State(U0, y0, l0, O.median3x3(l0, prm.height, prm.width), n0))
        bt.step()
        for s, (sv, prm, st) in enumerate(streams):
            _check_stream(bt, s, prm, starts2[s], f32(sv.frame(5)))


def test_graph_replay_is_bitwise_equal_to_launches():
    from paper_1302_2073_amd.tracker import BatchTracker
    streams = _streams(SHAPES[:3])
    res = []
    for graph in (False, True):
        with BatchTracker(_specs(streams)) as bt:
            bt.set_frames(_frames_tensor(streams, 4, 3))
            _load(bt, streams)
            bt.use_graph(graph)
            for _ in range(4):
                bt.step()
                assert bt.sync() == 0     # eager work between replays
            res.append([bt.get_state(s) for s in range(len(streams))])
    for a, b in zip(*res):
        for x, y in zip(a, b):
            assert np.array_equal(np.asarray(x), np.asarray(y))


def test_tuner_restores_state_and_keeps_parity(tmp_path):
    from paper_1302_2073_amd.tracker import BatchTracker
    streams = _streams(SHAPES[:4])
    with BatchTracker(_specs(streams)) as bt:
        bt.set_frames(_frames_tensor(streams, 4, 1))
        starts = _load(bt, streams)
        before = [bt.get_state(s) for s in range(len(streams))]
        rec = bt.tune(steps=2, cache=str(tmp_path / "tune.json"))
        say("  tuned", rec)
        after = [bt.get_state(s) for s in range(len(streams))]
        for a, b in zip(before, after):
            for x, y in zip(a, b):
                assert np.array_equal(np.asarray(x), np.asarray(y))
        bt.step()
        for s, (sv, prm, st) in enumerate(streams):
            _check_stream(bt, s, prm, starts[s], f32(sv.frame(4)))
        rec2 = bt.tune(steps=2, cache=str(tmp_path / "tune.json"))   # from the cache
        assert rec2["config"] == rec["config"]


@pytest.mark.parametrize("budget", [128, 192])
def test_batch_bf16_matches_oracle(budget):
    """bfloat16 batch against each stream's oracle step; budget 192 is the
    LDS form (row pairs of the tile held in LDS beside the registers)."""
    from paper_1302_2073_amd.tracker import BatchTracker

    def rne(a):
        f = np.asarray(a, np.float32)
        u = f.view(np.uint32).astype(np.uint64)
        return ((((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32)).view(np.float32).astype(np.float64)

    streams = _streams(SHAPES[:4])
    with BatchTracker(_specs(streams), storage="bf16") as bt:
        bt.configure(register_budget=budget, workgroups_per_cu=1)
        say("  config", bt.config())
        bt.set_frames(_frames_tensor(streams, 4, 1, "bf16"))
        starts = _load(bt, streams)
        bt.step()
        for s, (sv, prm, st) in enumerate(streams):
            x = rne(sv.frame(4))
            exp, _ = O.track_frame(starts[s], x, prm)
            U1, y1, l1, n1 = bt.get_state(s)
            y_rel = np.linalg.norm(y1 - exp.y) / np.linalg.norm(exp.y)
            e = rne(exp.U)
            ulp = np.exp2(np.floor(np.log2(np.maximum(np.abs(e), 1e-38))) - 7)
            ulp = ulp + update_rounding_bound(starts[s], x, prm, exp.y, y1)
            over = int(np.sum(np.abs(U1 - e) > ulp * 1.0000001 + 1e-45))
            say(f"  bf16 stream {s}: y {y_rel:.1e}, U entries beyond 1 ulp: {over}")
            assert y_rel <= 1e-4 and over == 0


def _rne(a):
    f = np.asarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    return ((((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32)).view(np.float32).astype(np.float64)


def _vga_bf16_frame(sv, n):
    import torch
    from paper_1302_2073_amd.tracker import bf16_bits
    return torch.from_numpy(bf16_bits(sv.frame(n)).view(np.int16)).cuda().view(torch.bfloat16)


def _vga_starts(bt, streams):
    starts = {}
    for s in streams:
        U0, y0, l0, n0 = bt.get_state(s)
        starts[s] = O.State(U0, y0, l0, O.median3x3(l0, 480, 640), n0)
    return starts


def _check_vga_bf16_step(bt, s, start, x, mu, prm=None):
    """One bfloat16 stream (640x480x3 k=15 unless prm says otherwise) after
    one step against its oracle step from the device's starting state: y
    within 1e-4, every U entry within one bfloat16 ulp of the
    round-to-nearest oracle value plus the float32 rounding bound of the
    update, labels exact outside the guard band."""
    prm = prm or O.Params(640, 480, 3, k=15, mu=mu)
    exp, _ = O.track_frame(start, x, prm)
    U1, y1, l1, n1 = bt.get_state(s)
    y_rel = np.linalg.norm(y1 - exp.y) / np.linalg.norm(exp.y)
    e = _rne(exp.U)
    ulp = np.exp2(np.floor(np.log2(np.maximum(np.abs(e), 1e-38))) - 7)
    ulp = ulp + update_rounding_bound(start, x, prm, exp.y, y1)
    over = int(np.sum(np.abs(U1 - e) > ulp * 1.0000001 + 1e-45))
    if over:
        r = (np.abs(U1 - e) / ulp).ravel()
        worst = np.argsort(r)[-5:]
        say("  worst entries (value, oracle, |diff|/bound):",
            [(float(U1.ravel()[i]), float(e.ravel()[i]), float(r[i])) for i in worst])
    band = O.band_pixels(exp.U, x, exp.y, prm.thr, prm.channels, GUARD)
    mism = int(np.sum((l1 != exp.labels) & ~band))
    say(f"  bf16 stream {s} {prm.width}x{prm.height}x{prm.channels} k={prm.k} n={start.n}: y {y_rel:.1e}, "
        f"U entries beyond 1 ulp: {over}, labels outside band {mism}")
    assert n1 == exp.n and y_rel <= 1e-4 and over == 0 and mism == 0
    assert np.array_equal(bt.mask(s), O.median3x3(l1, prm.height, prm.width))


@pytest.mark.parametrize("nstreams,budget,n0,threads", [(2, 0, 0, 512), (3, 192, 0, 512), (2, 0, 150, 512),
                                                         (2, 128, 0, 256), (2, 128, 150, 256)])
def test_batch_bf16_vga_streams_share_a_round(nstreams, budget, n0, threads):
    """640x480x3 k=15 streams in bfloat16 (the benchmark's streams): the
    row-pair tiles halve each gang, so two frames run side by side in one
    round, and three with the LDS form; each stream matches its own oracle
    step."""
    from paper_1302_2073_amd.tracker import BatchTracker

    wls = [V.vga_rgb(stream=s) for s in range(nstreams)]
    svs = [V.SyntheticVideo(w.video) for w in wls]
    specs = [dict(width=640, height=480, channels=3, k=15, mu=w.mu) for w in wls]
    with BatchTracker(specs, storage="bf16") as bt:
        if threads == 256:   # two 256-thread workgroups per CU, one of each stream
            bt.configure(register_budget=budget, workgroups_per_cu=2, threads=256)
        elif budget:
            bt.configure(register_budget=budget, workgroups_per_cu=1)
        cfg = bt.config()
        assert cfg["threads"] == threads
        say("  config", cfg)
        assert cfg["rounds"] == 1
        frames = [[_vga_bf16_frame(sv, 0)] for sv in svs]
        for s in range(nstreams):   # n0 = 150: past the initialization phase, t = t_min (Sec. 3.4)
            bt.set_state(s, V.initial_subspace(640 * 480 * 3, 15, 3, s), n=n0)
        bt.set_frames(frames)   # a ring of one frame: every step reads it whatever n is
        starts = _vga_starts(bt, range(nstreams))
        bt.step()
        assert bt.sync() == 0
        for s, w in enumerate(wls):
            _check_vga_bf16_step(bt, s, starts[s], _rne(svs[s].frame(0)), w.mu)


def test_benchmark_launch_configuration():
    """The benchmark's headline launch: 16 bfloat16 640x480x3 k=15 streams,
    register budget 128, one workgroup per CU, gangs in stream order (two
    per round, eight rounds), two-hop exchange, replayed from a hipGraph,
    32 steps per launch over a ring of 8 frames.  One step is checked
    against the oracle on a sample of streams from six of the eight rounds;
    then one 32-step launch must equal 32 single steps (no graph) bit for
    bit, for every stream's state and mask."""
    import hashlib
    from paper_1302_2073_amd.tracker import BatchTracker
    ns, ring = 16, 8
    wls = [V.vga_rgb(stream=s) for s in range(ns)]
    svs = [V.SyntheticVideo(w.video) for w in wls]
    specs = [dict(width=640, height=480, channels=3, k=15, mu=w.mu) for w in wls]
    frames = [[_vga_bf16_frame(sv, n) for n in range(ring)] for sv in svs]
    sample = [0, 3, 6, 9, 12, 15]

    def digest(bt):
        out = []
        for s in range(ns):
            U, y, lab, n = bt.get_state(s)
            out.append((hashlib.sha256(U.tobytes()).hexdigest(), y.tobytes(), lab.tobytes(), n,
                        bt.mask(s).tobytes()))
        return out

    res = []
    for multi in (True, False):
        with BatchTracker(specs, storage="bf16") as bt:
            bt.configure(register_budget=128, workgroups_per_cu=1, tile_scale=1.0, strategy=1, sync_mode=2)
            cfg = bt.config()
            say("  config", cfg)
            assert cfg["rounds"] == 8 and cfg["workgroups"] >= 226
            for s in range(ns):
                bt.set_state(s, V.initial_subspace(640 * 480 * 3, 15, 3, s))
            bt.set_frames(frames)
            bt.use_graph(multi)
            starts = _vga_starts(bt, sample) if multi else None
            bt.step()
            assert bt.sync() == 0
            if multi:
                for s in sample:
                    _check_vga_bf16_step(bt, s, starts[s], _rne(svs[s].frame(0)), wls[s].mu)
                bt.steps(32)
            else:
                for _ in range(32):
                    bt.step()
            assert bt.sync() == 0
            res.append(digest(bt))
    assert [r[3] for r in res[0]] == [33] * ns
    for s in range(ns):
        assert res[0][s] == res[1][s], f"stream {s}"


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_mixed_streams_workload_parity_sample(storage):
    """Four streams of the 64-stream mixed workload (one of each resolution
    plus the largest k) inside the full 64-stream launch, in float32 and in
    the workload's own bfloat16 storage."""
    from paper_1302_2073_amd.tracker import BatchTracker
    wls = V.mixed_streams(64)
    check = []
    seen = set()
    for i, wl in enumerate(wls):
        key = (wl.video.width, wl.k)
        if wl.video.width not in {w for w, _ in seen} or (wl.k == 15 and 15 not in {k for _, k in seen}):
            check.append(i)
            seen.add(key)
        if len(check) == 4:
            break
    specs = [dict(width=w.video.width, height=w.video.height, channels=3, k=w.k, mu=w.mu) for w in wls]
    import torch
    with BatchTracker(specs, storage=storage) as bt:
        say("  config", bt.config())
        frames = []
        svs = []
        for i, wl in enumerate(wls):
            sv = V.SyntheticVideo(wl.video)
            svs.append(sv)
            if storage == "f32":
                frames.append([torch.from_numpy(sv.frame(0).astype(np.float32)).cuda()])
            else:
                frames.append([_vga_bf16_frame(sv, 0)])
            bt.set_state(i, V.initial_subspace(wl.video.m, wl.k, 4, i))
        bt.set_frames(frames)
        starts = {}
        for i in check:
            U0, y0, l0, n0 = bt.get_state(i)
            starts[i] = O.State(U0, y0, l0, O.median3x3(l0, wls[i].video.height, wls[i].video.width), n0)
        bt.step()
        assert bt.sync() == 0
        for i in check:
            wl = wls[i]
            v = wl.video
            prm = O.Params(v.width, v.height, 3, k=wl.k, mu=wl.mu)
            if storage == "f32":
                _check_stream(bt, i, prm, starts[i], f32(svs[i].frame(0)))
            else:
                _check_vga_bf16_step(bt, i, starts[i], _rne(svs[i].frame(0)), wl.mu, prm)


@pytest.mark.parametrize("graph", [False, True])
def test_ordinary_dispatch_is_bitwise_equal(graph):
    """Ordinary launches (and their captured graph) give the same states as
    cooperative launches."""
    from paper_1302_2073_amd.tracker import BatchTracker
    streams = _streams(SHAPES[:3])
    res = []
    for coop in (1, 0):
        with BatchTracker(_specs(streams)) as bt:
            bt.set_dispatch(coop)
            bt.use_graph(graph)
            bt.set_frames(_frames_tensor(streams, 4, 2))
            _load(bt, streams)
            for _ in range(3):
                bt.step()
            assert bt.sync() == 0
            res.append([bt.get_state(s) for s in range(len(streams))])
    for sa, sb in zip(res[0], res[1]):
        for a, b in zip(sa, sb):
            np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("storage,budget", [("f32", 128), ("bf16", 128), ("bf16", 64)])
def test_multi_step_launch_is_bitwise_equal(storage, budget):
    """pros_batch_track_steps(b, 3) twice equals six single steps: each item
    keeps its tile in registers over three frames of its ring (register
    budget 128; at budget 64 the call falls back to one launch per step)."""
    from paper_1302_2073_amd.tracker import BatchTracker
    streams = _streams(SHAPES[:4])
    res = []
    for multi in (False, True):
        with BatchTracker(_specs(streams), storage=storage) as bt:
            bt.configure(register_budget=budget, workgroups_per_cu=1)
            bt.set_frames(_frames_tensor(streams, 4, 4, storage))
            _load(bt, streams)
            if multi:
                bt.steps(3)
                bt.steps(3)
            else:
                for _ in range(6):
                    bt.step()
            assert bt.sync() == 0
            res.append([bt.get_state(s) for s in range(len(streams))] +
                       [bt.mask(s) for s in range(len(streams))])
    say(f"  {storage}: n = {[int(st[3]) for st in res[1][:len(streams)]]}")
    for sa, sb in zip(res[0], res[1]):
        if isinstance(sa, tuple):
            for a, b in zip(sa, sb):
                np.testing.assert_array_equal(a, b)
        else:
            np.testing.assert_array_equal(sa, sb)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_256_thread_workgroups(storage):
    """Two 256-thread workgroups per CU (register budget 128, k class 15):
    every stream of an uneven batch matches its oracle step, and one 4-step
    launch equals four single steps bit for bit."""
    from paper_1302_2073_amd.tracker import BatchTracker
    streams = _streams(SHAPES[:3])
    res = []
    for multi in (False, True):
        with BatchTracker(_specs(streams), storage=storage) as bt:
            bt.configure(register_budget=128, workgroups_per_cu=2, threads=256)
            cfg = bt.config()
            say("  config", cfg)
            assert cfg["threads"] == 256 and cfg["workgroups"] >= 2 * 256 - 16
            bt.set_frames(_frames_tensor(streams, 4, 4, storage))
            starts = _load(bt, streams)
            if multi:
                bt.steps(4)
            else:
                bt.step()
                assert bt.sync() == 0
                for s, (sv, prm, st) in enumerate(streams):
                    if storage == "f32":
                        _check_stream(bt, s, prm, starts[s], f32(sv.frame(4)))
                    else:
                        _check_vga_bf16_step(bt, s, starts[s], _rne(sv.frame(4)), prm.mu, prm)
                for _ in range(3):
                    bt.step()
            assert bt.sync() == 0
            res.append([bt.get_state(s) for s in range(len(streams))] +
                       [bt.mask(s) for s in range(len(streams))])
    for sa, sb in zip(res[0], res[1]):
        if isinstance(sa, tuple):
            for a, b in zip(sa, sb):
                np.testing.assert_array_equal(a, b)
        else:
            np.testing.assert_array_equal(sa, sb)


def _per_call_state(storage, streams, rows, graph, ring_mode):
    """Six batch steps over frames rows[n][s] (n = step, s = stream), either
    registered as a ring of six (ring_mode) or handed over per call
    (pros_batch_track_frames); the final states and masks."""
    from paper_1302_2073_amd.tracker import BatchTracker
    with BatchTracker(_specs(streams), storage=storage) as bt:
        _load(bt, streams)
        bt.use_graph(graph)
        if ring_mode:   # stream s reads ring slot (frame counter) mod ring
            R = len(rows)
            n0 = [bt.get_state(s)[3] for s in range(len(streams))]
            bt.set_frames([[rows[(i - n0[s]) % R][s] for i in range(R)] for s in range(len(streams))])
            for _ in range(len(rows)):
                bt.step()
        else:
            for n in range(len(rows)):
                bt.track(rows[n])
        assert bt.sync() == 0
        return [bt.get_state(s) + (bt.mask(s),) for s in range(len(streams))]


@pytest.mark.parametrize("graph", [False, True])
def test_per_call_frames_equal_the_ring(graph):
    """pros_batch_track_frames (each call names that step's frames, the
    table updated in stream order from pinned staging) gives bit for bit the
    states and masks of stepping a registered ring over the same frames,
    with and without graph replay."""
    streams = _streams(SHAPES[:3], warm=2)
    fr = _frames_tensor(streams, 2, 6)
    rows = [[fr[s][n] for s in range(len(streams))] for n in range(6)]
    a = _per_call_state("f32", streams, rows, graph, ring_mode=True)
    b = _per_call_state("f32", streams, rows, graph, ring_mode=False)
    for s in range(len(streams)):
        for x, y in zip(a[s], b[s]):
            assert np.array_equal(np.asarray(x), np.asarray(y)), f"stream {s}"


def test_per_call_frames_with_changing_alignment():
    """bfloat16 frames handed over per call at alternating 4-byte and 2-byte
    aligned addresses (the calls whose alignment changes register the frames
    synchronously): the states follow the oracle step by step."""
    import torch
    streams = _streams([(64, 48, 3, 10), (80, 60, 1, 5)], warm=2)
    fr = _frames_tensor(streams, 2, 4, "bf16")
    from paper_1302_2073_amd.tracker import BatchTracker, bf16_to_f64
    with BatchTracker(_specs(streams), storage="bf16") as bt:
        starts = _load(bt, streams)
        keep = []
        for n in range(4):
            row = []
            for s in range(len(streams)):
                t = fr[s][n]
                if n % 2 == 1:   # an odd bfloat16 offset: not 4-byte aligned
                    buf = torch.empty(t.numel() + 1, dtype=torch.bfloat16, device="cuda")
                    buf[1:].copy_(t)
                    t = buf[1:]
                row.append(t)
            keep.append(row)
            bt.track(row)
            assert bt.sync() == 0
            nxt = []
            for s, (sv, prm, _) in enumerate(streams):
                x64 = bf16_to_f64(fr[s][n].cpu().view(torch.int16).numpy().view(np.uint16))
                exp, _ = O.track_frame(starts[s], x64, prm)
                U1, y1, l1, n1 = bt.get_state(s)
                assert n1 == exp.n
                assert np.linalg.norm(y1 - exp.y) / np.linalg.norm(exp.y) <= TOL_Y
                band = O.band_pixels(exp.U, x64, exp.y, prm.thr, prm.channels, GUARD)
                assert int(np.sum((l1 != exp.labels) & ~band)) == 0
                nxt.append(O.State(U1, y1, l1, O.median3x3(l1, prm.height, prm.width), n1))
            starts = nxt


def test_batch_refuses_streams_beyond_the_resident_tiles():
    """A stream whose gang of register tiles cannot be resident (1280x720x3
    at k = 15, which a single tracker runs in its streamed form) is refused
    by pros_batch_init with PROS_EUNSUPPORTED, and per-call frames with a NULL
    pointer are refused with PROS_EINVAL, before any launch."""
    from paper_1302_2073_amd import _lib as L
    from paper_1302_2073_amd.tracker import BatchTracker
    with pytest.raises(L.ProstError) as ei:
        BatchTracker([dict(width=1280, height=720, channels=3, k=15, mu=1e-3)], storage="f32")
    assert ei.value.status == L.PROS_EUNSUPPORTED
    import ctypes as C
    with BatchTracker([dict(width=80, height=60, channels=1, k=5, mu=1e-3)], storage="f32") as bt:
        ptrs = (C.c_void_p * 1)()
        assert L.lib().pros_batch_track_frames(bt._b, ptrs) == L.PROS_EINVAL
