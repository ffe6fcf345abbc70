"""Batched detection (many uneven frames in one launch sequence, graph replay, tuning) against
per-frame detection on the GPU, and against the oracle."""
import sys

import numpy as np
import pytest
import torch

from oracle import ridge_hough as O
from paper_1310_1371_amd import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _frames_u16():
    """Four uint16 frames of uneven sizes with the x1000-count ring model."""
    out = []
    for i, (W, H, n) in enumerate(((300, 170, 12), (512, 512, 60), (640, 480, 80), (1024, 768, 150))):
        f = synth.config2(seed=300 + i, W=W, H=H, n_rings=n)
        out.append(f)
    return out


@pytest.fixture(scope="module")
def bdet():
    from paper_1310_1371_amd.detector import Detector
    d = Detector(max_width=2048, max_height=2048, max_peaks=16384, max_frames=8,
                 max_batch_pixels=8 * 2048 * 1088)
    yield d
    d.close()


def _same(a, b):
    return a.tobytes() == b.tobytes()


def test_batch_equals_per_frame(bdet):
    say("[batch] 4 uneven u16 frames vs per-frame")
    fs = _frames_u16()
    p = fs[0].params
    frames = [torch.from_numpy(f.image).cuda() for f in fs]
    batch = bdet.detect_batch(frames, p)
    for f, fr, got in zip(fs, frames, batch):
        ref = bdet.detect(fr, p)
        assert _same(ref, got), (f.image.shape, len(ref), len(got))
        say(f"  {f.image.shape}: {len(got)} rings")


def test_rings_come_out_sorted(bdet):
    say("[batch] every frame's rings in strictly ascending (r_bin, b, a) order")
    fs = _frames_u16()
    frames = [torch.from_numpy(f.image).cuda() for f in fs]
    for rings in bdet.detect_batch(frames, fs[0].params):
        keys = [(int(r["r_bin"]), int(r["b"]), int(r["a"])) for r in rings]
        assert len(keys) >= 5
        assert all(k0 < k1 for k0, k1 in zip(keys, keys[1:]))


def test_edge_batch_equals_per_frame_and_modes_alternate(bdet):
    """Directed edges through the batched path equal per-frame edge detections, and
    alternating the measure between calls (each a different captured graph) gives each
    mode's own rings back unchanged."""
    say("[batch] directed edges: 4 uneven u16 frames vs per-frame, modes alternating")
    fs = _frames_u16()
    p_ridge = fs[0].params
    p_edge = dict(p_ridge, measure=1, k_threshold=-12.0)
    frames = [torch.from_numpy(f.image).cuda() for f in fs]
    ridge0 = bdet.detect_batch(frames, p_ridge)
    edge0 = bdet.detect_batch(frames, p_edge)
    for f, fr, got in zip(fs, frames, edge0):
        ref = bdet.detect(fr, p_edge)
        assert _same(ref, got), (f.image.shape, len(ref), len(got))
        say(f"  {f.image.shape}: {len(got)} edge rings")
    ridge1 = bdet.detect_batch(frames, p_ridge)
    edge1 = bdet.detect_batch(frames, p_edge)
    assert all(_same(a, b) for a, b in zip(ridge0, ridge1))
    assert all(_same(a, b) for a, b in zip(edge0, edge1))
    assert any(not _same(a, b) for a, b in zip(ridge0, edge0))


def test_batch_graph_replay_uses_new_data(bdet):
    say("[batch] graph replay with new frame contents")
    bdet.set_tuning(use_graph=True)
    fs = _frames_u16()
    p = fs[0].params
    bufs = [torch.from_numpy(f.image).cuda() for f in fs]
    first = bdet.detect_batch(bufs, p)
    again = bdet.detect_batch(bufs, p)
    assert all(_same(a, b) for a, b in zip(first, again))
    # same shapes, different contents, same device buffers: the replayed graph must see them
    fs2 = [synth.config2(seed=400 + i, W=f.width, H=f.height, n_rings=40) for i, f in enumerate(fs)]
    for buf, f in zip(bufs, fs2):
        buf.copy_(torch.from_numpy(f.image).cuda())
    torch.cuda.synchronize()
    replay = bdet.detect_batch(bufs, p)
    bdet.set_tuning(use_graph=False)
    direct = bdet.detect_batch(bufs, p)
    bdet.set_tuning(use_graph=True)
    for a, b, f in zip(replay, direct, fs2):
        assert _same(a, b)
    # and they agree with the oracle on a small frame
    ref = O.detect(fs2[0].image, p)
    kr = {(int(r["a"]), int(r["b"]), int(r["r_bin"])) for r in ref}
    kg = {(int(r["a"]), int(r["b"]), int(r["r_bin"])) for r in replay[0]}
    assert len(kr ^ kg) <= max(1, 0.01 * len(kr))


def test_batch_host_frames(bdet):
    say("[batch] host frames")
    fs = _frames_u16()[:2]
    p = fs[0].params
    host = bdet.detect_batch([f.image for f in fs], p)
    dev = bdet.detect_batch([torch.from_numpy(f.image).cuda() for f in fs], p)
    assert all(_same(a, b) for a, b in zip(host, dev))


@pytest.mark.parametrize("stencil_tile", [0, 1, 2])
@pytest.mark.parametrize("vote_lds_kb", [24, 44, None])
def test_tuning_invariance(bdet, stencil_tile, vote_lds_kb):
    say(f"[tuning] stencil {stencil_tile} lds {vote_lds_kb}")
    f = synth.config2(seed=77, W=640, H=480, n_rings=80)
    img = torch.from_numpy(f.image).cuda()
    bdet.set_tuning(stencil_tile=0, use_graph=True)
    ref = bdet.detect(img, f.params)
    xy0, q0, _ = bdet.ridges(img, f.params)
    bdet.set_tuning(stencil_tile=stencil_tile, vote_lds_kb=vote_lds_kb, use_graph=True)
    got = bdet.detect(img, f.params)
    xy1, q1, _ = bdet.ridges(img, f.params)
    bdet.set_tuning(stencil_tile=0, use_graph=True)
    assert _same(ref, got)
    s0 = set(map(tuple, torch.cat([xy0, q0.int()], 1).cpu().numpy().tolist()))
    s1 = set(map(tuple, torch.cat([xy1, q1.int()], 1).cpu().numpy().tolist()))
    assert s0 == s1


def test_timing_events_inside_the_graph(bdet):
    """With timing on, the replayed graph carries the event records: every stage is timed on
    every call, and the rings stay the same with timing on, and after it is turned off."""
    say("[timing] events as graph nodes")
    f = synth.config2(seed=78, W=640, H=480, n_rings=80)
    img = torch.from_numpy(f.image).cuda()
    bdet.set_tuning(use_graph=True)
    ref = bdet.detect(img, f.params)
    bdet.enable_timing(True)
    bdet.read_timing(reset=True)
    for _ in range(3):
        assert _same(ref, bdet.detect(img, f.params))
    t = bdet.read_timing(reset=True)
    bdet.enable_timing(False)
    # the first call of every eight is timed
    assert all(n == 1 for _, n in t.values()), t
    assert all(ms > 0.0 for ms, _ in t.values()), t
    assert _same(ref, bdet.detect(img, f.params))


def test_tuning_beyond_the_lds_limit_is_rejected(bdet):
    """The default is the largest histogram budget; one KiB more is refused on the host."""
    top = bdet.default_tuning["vote_lds_kb"]
    assert bdet.get_tuning()["vote_lds_kb"] == top
    from paper_1310_1371_amd.native import RdError
    with pytest.raises(RdError):
        bdet.set_tuning(vote_lds_kb=top + 1)
    with pytest.raises(RdError):
        bdet.set_tuning(vote_lds_kb=15)
    assert bdet.get_tuning()["vote_lds_kb"] == top


@pytest.mark.parametrize("vote_lds_kb", [16, 32])
def test_accumulator_invariant_to_level_chunks(bdet, vote_lds_kb):
    say(f"[tuning] accumulator with lds {vote_lds_kb}")
    f = synth.config1()
    p = dict(O.DEFAULTS, **f.params)
    xs, ys, qx, qy, _ = O.ridges(f.image, p)
    xy = np.stack([xs, ys], 1).astype(np.int32)
    q = np.stack([qx, qy], 1).astype(np.int16)
    bdet.set_tuning()
    a0, s0 = bdet.accumulate(xy, q, 256, 256, p)
    bdet.set_tuning(vote_lds_kb=vote_lds_kb)
    a1, s1 = bdet.accumulate(xy, q, 256, 256, p)
    bdet.set_tuning()
    assert torch.equal(a0, a1) and torch.equal(s0, s1)


def test_autotune_returns_a_valid_choice(bdet):
    say("[tuning] autotune")
    fs = _frames_u16()[:2]
    t = bdet.autotune([torch.from_numpy(f.image).cuda() for f in fs], fs[0].params, reps=1)
    assert t["stencil_tile"] in (0, 1, 2) and 16 <= t["vote_lds_kb"] <= bdet.default_tuning["vote_lds_kb"]
    bdet.set_tuning(stencil_tile=0, use_graph=True)


def test_batch_limits(bdet):
    say("[batch] limits")
    from paper_1310_1371_amd import native as N
    f = synth.config1()
    with pytest.raises(N.RdError) as e:
        bdet.detect_batch([f.image] * 9, f.params)
    assert e.value.status == N.RD_E_TOO_LARGE
    with pytest.raises(N.RdError) as e:
        bdet.detect_batch([f.image, f.image.astype(np.uint16)], f.params)
    assert e.value.status == N.RD_E_INVALID


def test_stats_counts(bdet):
    say("[stats]")
    f = synth.config1()
    rings = bdet.detect(torch.from_numpy(f.image).cuda(), f.params)
    st = bdet.stats()
    xs, ys, qx, qy, _ = O.ridges(f.image, f.params)
    assert st["peaks"] == len(rings)
    assert abs(st["ridges"] - len(xs)) <= max(1, 1e-4 * len(xs))
    assert st["votes"] > 0 and st["hotspots"] > 0 and st["strong"] >= st["peaks"]


def test_vote_profiles(bdet):
    """The profiling instance of the vote kernel: the same rings as the plain call, phase clocks
    over every tile, and one record per vote tile (each queue position once, the ridge tiles
    of 40 px, every workgroup below the CU count, end after start)."""
    say("[vote profiles]")
    f = synth.config2(seed=21, W=300, H=170, n_rings=12)
    img = torch.from_numpy(f.image).cuda()
    ref = bdet.detect(img, f.params)
    ph = bdet.profile_vote_phases(img, f.params)
    tiles = ((300 + 39) // 40) * ((170 + 39) // 40)
    assert ph["tiles"] == tiles and all(v > 0 for v in ph["phases"].values())
    assert ph["lifetime_min"] <= ph["lifetime_max"]
    rec = bdet.profile_vote_tiles(img, f.params)
    assert rec.shape == (tiles, 4)
    assert sorted(rec[:, 1].tolist()) == list(range(tiles))
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert (rec[:, 0] >= 0).all() and (rec[:, 0] < cus).all() and (rec[:, 3] > rec[:, 2]).all()
    assert bdet.detect(img, f.params).tobytes() == ref.tobytes()
    # a record buffer short of the frame's tiles: RD_E_TRUNCATED with the count, nothing written
    import ctypes
    from paper_1310_1371_amd import native as N
    from paper_1310_1371_amd.detector import _frame_struct
    buf = np.full(4 * (tiles - 1), 7, dtype=np.uint64)
    n = ctypes.c_int32(0)
    st = N.lib().rd_profile_vote_tiles(bdet._h, ctypes.byref(_frame_struct(img)), ctypes.byref(N.make_params(f.params)),
                                       buf.ctypes.data_as(ctypes.c_void_p), tiles - 1, ctypes.byref(n))
    assert st == N.RD_E_TRUNCATED and n.value == tiles and (buf == 7).all()
