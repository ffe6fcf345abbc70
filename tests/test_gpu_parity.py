"""GPU (HIP, through the C ABI) against the FP64 CPU oracle, stage by stage and end to end.

Tolerances: k_- within 1e-5 relative with a floor of 1e-3 of the frame's largest |k_-|;
direction codes exact except +/-1 flips at rounding ties (counted); ridge sets within 0.01 %
of the oracle's ridge count (counted); vote accumulators and integer scores bit-exact when
fed the oracle's ridges; rings within 0.05 px in centre and radius."""
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


@pytest.fixture(scope="module")
def det():
    from paper_1310_1371_amd.detector import Detector
    d = Detector(max_width=2048, max_height=2048, max_peaks=65536)
    yield d
    d.close()


def _ragged():
    """300 x 170 uint16 frame (not a multiple of any tile size), c2-like content."""
    f = synth.config2(seed=21, W=300, H=170, n_rings=12)
    return f


def _tail():
    """161 x 97 float32, one column and one row past a multiple of 32 px (and a column past a
    multiple of the 40 px vote tile), with rings centred on the last column and the last row:
    the last tiles' score regions are one or two pixels wide."""
    cx, cy, R = np.array([160.0, 80.0]), np.array([48.0, 96.0]), np.array([20.0, 15.0])
    s, A = np.full(2, 1.5), np.ones(2)
    img = synth.render(161, 97, np.zeros((97, 161)), cx, cy, R, s, A)
    return synth.Frame(img.astype(np.float32), cx, cy, R, s, A, dict(synth.PARAMS_C1), 0)


def _tail40():
    """121 x 81 float32, one column and one row past a multiple of the 40 px vote tile, with
    rings centred on the last column and the last row."""
    cx, cy, R = np.array([120.0, 60.0]), np.array([30.0, 80.0]), np.array([18.0, 14.0])
    s, A = np.full(2, 1.5), np.ones(2)
    img = synth.render(121, 81, np.zeros((81, 121)), cx, cy, R, s, A)
    return synth.Frame(img.astype(np.float32), cx, cy, R, s, A, dict(synth.PARAMS_C1), 0)


def _big_ring():
    """300 x 300 float32 with one ring of radius 123 px and radius bins 100-126 (the largest
    r_max): the fit visits 17 x 17 ridge bins, more than one round of the fit's bin list."""
    f = synth.single_ring(300, 300, 150.3, 149.6, 123.0)
    return synth.Frame(f.image, f.cx, f.cy, f.R, f.s, f.A, dict(f.params, r_min=100, r_max=126), 0)


def _concentric():
    """300 x 300 float32 with 15 concentric rings (radii 10, 14, ..., 66 px, one centre) and
    radius bins 8-70: one tile's level chunks hold up to 208 above-threshold voxels, past the
    64 at which the 3x3x3 test looks neighbours up in a hash table."""
    R = 10.0 + 4.0 * np.arange(15)
    k = len(R)
    cx, cy = np.full(k, 150.3), np.full(k, 149.6)
    s, A = np.full(k, 1.5), np.ones(k)
    img = synth.render(300, 300, np.zeros((300, 300)), cx, cy, R, s, A)
    return synth.Frame(img.astype(np.float32), cx, cy, R, s, A, dict(synth.PARAMS_C1, r_max=70), 0)


CASES = {
    "c1_256_f32": lambda: synth.config1(),
    "ragged_300x170_u16": _ragged,
    "min_32x32_f32": lambda: synth.single_ring(32, 32, 15.0, 16.0, 9.3),
    "tail_161x97_f32": _tail,
    "tail_121x81_f32": _tail40,
    "big_ring_300_f32": _big_ring,
    "concentric_300_f32": _concentric,
}


def _frame(name):
    f = CASES[name]()
    return f


def _ktol(k_ref):
    return 1e-5 * np.maximum(np.abs(k_ref), 1e-3 * np.abs(k_ref).max())


def _check_curvature(det, f):
    p = f.params
    k_ref, qx_ref, qy_ref = O.curvature(f.image.astype(np.float64), O.f32(p["sigma_smooth"]))
    k, q = det.curvature(torch.from_numpy(f.image).cuda(), p)
    k = k.cpu().numpy().astype(np.float64)
    q = q.cpu().numpy().astype(np.int64)
    err = np.abs(k - k_ref)
    assert np.all(err <= _ktol(k_ref)), float((err / _ktol(k_ref)).max())
    # X_- is only defined where the eigenvalues differ: at (near-)isotropic points, where the
    # eigengap 2d is within rounding of the smoothed input, any direction is as good
    Ixx, Iyy, Ixy = O.hessian(f.image.astype(np.float64), O.f32(p["sigma_smooth"]))
    d = np.hypot(0.5 * (Ixx - Iyy), Ixy)
    defined = d > 1e-9 * np.abs(f.image).max()
    dqx, dqy = np.abs(q[..., 0] - qx_ref), np.abs(q[..., 1] - qy_ref)
    flips = int((((dqx > 0) | (dqy > 0)) & defined).sum())
    say(f"  k max rel err {float((err / np.maximum(np.abs(k_ref), 1e-300)).max()):.2e}; "
        f"q flips {flips}; isotropic pixels {int((~defined).sum())}")
    assert max(dqx[defined].max(), dqy[defined].max()) <= 1
    assert flips <= max(1, 1e-5 * k.size)


@pytest.mark.parametrize("name", list(CASES))
def test_curvature_parity(det, name):
    say(f"[curvature] {name}")
    _check_curvature(det, _frame(name))


def test_curvature_parity_c2_full(det):
    say("[curvature] c2 1024x1024 u16")
    _check_curvature(det, synth.config2())


def test_curvature_host_frame_and_pitch(det):
    say("[curvature] host frame and padded pitch")
    f = synth.config1()
    k_dev, q_dev = det.curvature(torch.from_numpy(f.image).cuda(), f.params)
    k_host, q_host = det.curvature(f.image, f.params)
    assert torch.equal(k_dev, k_host) and torch.equal(q_dev, q_host)
    padded = torch.zeros((256, 300), dtype=torch.float32, device="cuda")
    padded[:, :256] = torch.from_numpy(f.image).cuda()
    k_pad, q_pad = det.curvature(padded[:, :256], f.params)
    assert torch.equal(k_dev, k_pad) and torch.equal(q_dev, q_pad)


def _ridge_sets(det, f):
    p = f.params
    xs, ys, qx, qy, kk = O.ridges(f.image, p)
    xy, q, k = det.ridges(torch.from_numpy(f.image).cuda(), p)
    xy = xy.cpu().numpy().astype(np.int64)
    q = q.cpu().numpy().astype(np.int64)
    ref = {(int(x), int(y)): (int(a), int(b)) for x, y, a, b in zip(xs, ys, qx, qy)}
    got = {(int(x), int(y)): (int(a), int(b)) for (x, y), (a, b) in zip(xy, q)}
    return ref, got, len(xy)


@pytest.mark.parametrize("name", ["c1_256_f32", "ragged_300x170_u16"])
def test_ridge_parity(det, name):
    say(f"[ridges] {name}")
    f = _frame(name)
    ref, got, n = _ridge_sets(det, f)
    assert n == len(got), "duplicate ridge pixels"
    sym = set(ref) ^ set(got)
    say(f"  oracle {len(ref)} gpu {len(got)} mismatched {len(sym)}")
    assert len(sym) <= max(0, int(1e-4 * len(ref)))
    for key in set(ref) & set(got):
        assert max(abs(ref[key][0] - got[key][0]), abs(ref[key][1] - got[key][1])) <= 1


def test_ridge_parity_c2_full(det):
    say("[ridges] c2 1024x1024 u16")
    f = synth.config2()
    ref, got, n = _ridge_sets(det, f)
    sym = set(ref) ^ set(got)
    say(f"  oracle {len(ref)} gpu {len(got)} mismatched {len(sym)} ({100.0 * len(sym) / len(ref):.4f} %)")
    assert len(sym) <= 1e-4 * len(ref)


def _oracle_ridge_inputs(f):
    xs, ys, qx, qy, _ = O.ridges(f.image, f.params)
    xy = np.stack([xs, ys], 1).astype(np.int32)
    q = np.stack([qx, qy], 1).astype(np.int16)
    return xs, ys, qx, qy, xy, q


@pytest.mark.parametrize("name", ["c1_256_f32", "ragged_300x170_u16", "min_32x32_f32", "tail_161x97_f32", "tail_121x81_f32",
                                  "big_ring_300_f32", "concentric_300_f32"])
def test_accumulator_and_scores_bit_exact(det, name):
    say(f"[accumulate] {name}")
    f = _frame(name)
    p = dict(O.DEFAULTS, **f.params)
    H, W = f.image.shape
    xs, ys, qx, qy, xy, q = _oracle_ridge_inputs(f)
    rings_ref, A_ref, S_ref = O.detect_from_ridges(xs, ys, qx, qy, W, H, p, return_volumes=True)
    acc, sc = det.accumulate(xy, q, W, H, p)
    np.testing.assert_array_equal(acc.cpu().numpy().astype(np.int64), A_ref)
    np.testing.assert_array_equal(sc.cpu().numpy(), S_ref)


def test_dense_ridges_pieces_and_per_level_hotspots(det):
    """A 120 x 120 block in which every pixel is a ridge with a random direction (14400 ridges,
    full 16 x 16 bins): each vote tile sees several times more candidate ridges than it stages
    at once, and with T_int = 0 more hotspots per level chunk than its list holds, so both
    fallbacks (ridges staged in pieces, hotspots listed level by level) run."""
    say("[accumulate] dense ridge block, T_int = 0")
    W = H = 160
    yy, xx = np.mgrid[20:140, 20:140]
    xs, ys = xx.ravel().astype(np.int64), yy.ravel().astype(np.int64)
    th = np.random.default_rng(7).uniform(0.0, 2.0 * np.pi, xs.size)
    qx, qy = O.direction_code(np.cos(th), np.sin(th))
    p = dict(O.DEFAULTS, **dict(synth.PARAMS_C1, vote_threshold=0, peak_fraction=50.0))
    _, A_ref, S_ref = O.detect_from_ridges(xs, ys, qx, qy, W, H, p, return_volumes=True)
    xy = np.stack([xs, ys], 1).astype(np.int32)
    q = np.stack([qx, qy], 1).astype(np.int16)
    acc, sc = det.accumulate(xy, q, W, H, p)
    np.testing.assert_array_equal(acc.cpu().numpy().astype(np.int64), A_ref)
    np.testing.assert_array_equal(sc.cpu().numpy(), S_ref)


def test_strong_list_overflow_is_reported(det):
    """The same dense block with every hotspot above the score threshold overflows the per-chunk
    list of above-threshold voxels: the call reports RD_E_OVERFLOW instead of a wrong answer."""
    from paper_1310_1371_amd import native as N
    say("[accumulate] strong-list overflow")
    yy, xx = np.mgrid[20:140, 20:140]
    xs, ys = xx.ravel(), yy.ravel()
    th = np.random.default_rng(7).uniform(0.0, 2.0 * np.pi, xs.size)
    xy = np.stack([xs, ys], 1).astype(np.int32)
    q = np.stack(O.direction_code(np.cos(th), np.sin(th)), 1).astype(np.int16)
    p = dict(O.DEFAULTS, **dict(synth.PARAMS_C1, vote_threshold=0, peak_fraction=0.0))
    with pytest.raises(N.RdError) as e:
        det.accumulate(xy, q, 160, 160, p)
    assert e.value.status == N.RD_E_OVERFLOW


def _crowded(peak_fraction, vote_threshold):
    """256 x 256 float32 with six rings of radius 72.6-80.5 px whose centres all lie in the vote
    tile x, y in [96, 128), radius bins 8-80: at f = 0.25 that tile holds about 1100
    above-threshold voxels at radii 72-81 (about 110 per level), at f = 0.15 about 150 per
    level, both beyond the 512 of one level chunk's list, so the 3x3x3 test runs over windows
    of peak levels (several levels, then one level per window).  Such tiles occur in the
    2048^2 stream when two large rings' centres meet."""
    cx = np.array([108.3, 113.6, 104.2, 116.9, 110.1, 119.4])
    cy = np.array([110.8, 116.4, 118.1, 106.7, 104.5, 118.9])
    R = np.array([74.2, 77.4, 79.3, 75.8, 72.6, 80.5])
    s, A = np.full(6, 1.5), np.ones(6)
    img = synth.render(256, 256, np.full((256, 256), 0.2), cx, cy, R, s, A).astype(np.float32)
    p = dict(O.DEFAULTS, **dict(synth.PARAMS_C1, r_min=8, r_max=80, peak_fraction=peak_fraction,
                                vote_threshold=vote_threshold))
    return img, p


@pytest.mark.parametrize("f,tint", [(0.25, 3), (0.15, 2)])
def test_crowded_tile_windows_exact(det, f, tint):
    say(f"[crowded tile] f = {f}, T_int = {tint}")
    img, p = _crowded(f, tint)
    H, W = img.shape
    xs, ys, qx, qy, _ = O.ridges(img, p)
    ref, A_ref, S_ref = O.detect_from_ridges(xs, ys, qx, qy, W, H, p, return_volumes=True)
    lbase = p["r_min"] - 1
    thr = np.array([O.score_threshold(lbase + i, p) for i in range(S_ref.shape[0])])
    n_strong = int((S_ref > thr[:, None, None])[72 - lbase:82 - lbase, 95:129, 95:129].sum())
    say(f"  strong voxels of the tile at radii 72-81: {n_strong}; oracle rings {len(ref)}")
    assert n_strong > 2 * 512                      # the case does exercise the windows
    xy = np.stack([xs, ys], 1).astype(np.int32)
    q = np.stack([qx, qy], 1).astype(np.int16)
    acc, sc = det.accumulate(xy, q, W, H, p)
    np.testing.assert_array_equal(acc.cpu().numpy().astype(np.int64), A_ref)
    np.testing.assert_array_equal(sc.cpu().numpy(), S_ref)
    got = det.detect_from_ridges(xy, q, W, H, p)
    assert [tuple(int(v) for v in (r["a"], r["b"], r["r_bin"])) for r in ref] == \
           [tuple(int(v) for v in (r["a"], r["b"], r["r_bin"])) for r in got]
    np.testing.assert_array_equal(ref["n_fit"], got["n_fit"])
    np.testing.assert_array_equal(ref["fit_ok"], got["fit_ok"])
    for fld in ("cx", "cy", "r", "score"):
        np.testing.assert_allclose(got[fld], ref[fld], rtol=2e-7, atol=1e-9)
    # end to end from the frame
    e2e = det.detect(torch.from_numpy(img).cuda(), p)
    kr, kg = _match(O.detect(img, p), e2e)
    assert len(set(kr) ^ set(kg)) <= max(1, 0.01 * len(kr))
    for k in set(kr) & set(kg):
        for fld in ("cx", "cy", "r"):
            assert abs(float(kr[k][fld]) - float(kg[k][fld])) <= 0.05


def _dense_rings(tint):
    """40 rings of radius 6-28 on a 200^2 frame (radii 5-30): about 3600 ridges."""
    rng = np.random.default_rng(5)
    k = 40
    cx, cy, R = rng.uniform(20, 180, k), rng.uniform(20, 180, k), rng.uniform(6, 28, k)
    img = synth.render(200, 200, np.full((200, 200), 0.2), cx, cy, R, np.full(k, 1.5), np.ones(k))
    p = dict(O.DEFAULTS, **dict(synth.PARAMS_C1, r_min=5, r_max=30, vote_threshold=tint))
    return img.astype(np.float32), p


def test_per_level_hotspots_with_handed_over_levels(det):
    """With T_int = 0 a tile lists more hotspots in a level chunk after its first than the list
    holds (over 1792 at levels 20-27), so that chunk lists its hotspots level by level, while
    the strong voxels stay few (no window): the chunk takes its two bottom levels from the
    strong voxels the previous chunk handed over, also in the level-by-level listing.  Rings
    equal the oracle's from the same ridges."""
    say("[per-level hotspots after a hand-over] 200^2, 40 rings, T_int = 0")
    img, p = _dense_rings(0)
    H, W = img.shape
    xs, ys, qx, qy, _ = O.ridges(img, p)
    ref, A_ref, S_ref = O.detect_from_ridges(xs, ys, qx, qy, W, H, p, return_volumes=True)
    lbase = p["r_min"] - 1
    thr = np.array([O.score_threshold(lbase + i, p) for i in range(S_ref.shape[0])])
    strong = S_ref > thr[:, None, None]
    region = [(max(y - 1, 0), y + 41, max(x - 1, 0), x + 41) for y in range(0, H, 40) for x in range(0, W, 40)]
    hot_late = max(int((A_ref[20:, y0:y1, x0:x1] > 0).sum()) for y0, y1, x0, x1 in region)
    most_strong = max(int(strong[:, y0:y1, x0:x1].sum()) for y0, y1, x0, x1 in region)
    say(f"  most hotspots of a tile at levels 20-27: {hot_late}; most strong voxels of a tile: {most_strong}")
    assert hot_late > 1792 and most_strong < 512    # the case does exercise that path
    xy = np.stack([xs, ys], 1).astype(np.int32)
    q = np.stack([qx, qy], 1).astype(np.int16)
    got = det.detect_from_ridges(xy, q, W, H, p)
    assert [tuple(int(v) for v in (r["a"], r["b"], r["r_bin"])) for r in ref] == \
           [tuple(int(v) for v in (r["a"], r["b"], r["r_bin"])) for r in got]
    np.testing.assert_array_equal(ref["n_fit"], got["n_fit"])
    np.testing.assert_array_equal(ref["fit_ok"], got["fit_ok"])
    for fld in ("cx", "cy", "r", "score"):
        np.testing.assert_allclose(got[fld], ref[fld], rtol=2e-7, atol=1e-9)


def test_crowded_tile_overflow_reported(det):
    """With f = 0.1 and T_int = 1 a window of one peak level (three levels) holds more
    above-threshold voxels than the list: RD_E_OVERFLOW, not a partial answer."""
    from paper_1310_1371_amd import native as N
    say("[crowded tile] f = 0.1, T_int = 1: overflow")
    img, p = _crowded(0.1, 1)
    xs, ys, qx, qy, _ = O.ridges(img, p)
    xy = np.stack([xs, ys], 1).astype(np.int32)
    q = np.stack([qx, qy], 1).astype(np.int16)
    with pytest.raises(N.RdError) as e:
        det.detect_from_ridges(xy, q, 256, 256, p)
    assert e.value.status == N.RD_E_OVERFLOW


def test_accumulator_bit_exact_c2_full(det):
    say("[accumulate] c2 1024x1024, 68 levels")
    f = synth.config2()
    p = dict(O.DEFAULTS, **f.params)
    H, W = f.image.shape
    xs, ys, qx, qy, xy, q = _oracle_ridge_inputs(f)
    A_ref = O.vote(xs, ys, qx, qy, W, H, p["r_min"] - 1, p["r_max"] + 1)
    acc, _ = det.accumulate(xy, q, W, H, p, scores=False)
    assert torch.equal(acc.cpu().to(torch.int64), torch.from_numpy(A_ref))


def _match(ref, got):
    kr = {(int(r["a"]), int(r["b"]), int(r["r_bin"])): r for r in ref}
    kg = {(int(r["a"]), int(r["b"]), int(r["r_bin"])): r for r in got}
    return kr, kg


@pytest.mark.parametrize("name", ["c1_256_f32", "ragged_300x170_u16", "min_32x32_f32", "tail_161x97_f32", "tail_121x81_f32",
                                  "big_ring_300_f32", "concentric_300_f32"])
def test_rings_from_oracle_ridges_exact(det, name):
    say(f"[rings from oracle ridges] {name}")
    f = _frame(name)
    p = dict(O.DEFAULTS, **f.params)
    H, W = f.image.shape
    xs, ys, qx, qy, xy, q = _oracle_ridge_inputs(f)
    ref = O.detect_from_ridges(xs, ys, qx, qy, W, H, p)
    got = det.detect_from_ridges(xy, q, W, H, p)
    assert [tuple(int(v) for v in (r["a"], r["b"], r["r_bin"])) for r in ref] == \
           [tuple(int(v) for v in (r["a"], r["b"], r["r_bin"])) for r in got]
    np.testing.assert_array_equal(ref["n_fit"], got["n_fit"])
    np.testing.assert_array_equal(ref["fit_ok"], got["fit_ok"])
    for fld in ("cx", "cy", "r", "score"):
        np.testing.assert_allclose(got[fld], ref[fld], rtol=2e-7, atol=1e-9)


def test_rings_from_oracle_ridges_c2_full(det):
    say("[rings from oracle ridges] c2 1024x1024")
    f = synth.config2()
    p = dict(O.DEFAULTS, **f.params)
    H, W = f.image.shape
    xs, ys, qx, qy, xy, q = _oracle_ridge_inputs(f)
    ref = O.detect_from_ridges(xs, ys, qx, qy, W, H, p)
    got = det.detect_from_ridges(xy, q, W, H, p)
    say(f"  oracle {len(ref)} rings, gpu {len(got)}")
    assert len(ref) == len(got)
    np.testing.assert_array_equal(ref["a"], got["a"])
    np.testing.assert_array_equal(ref["r_bin"], got["r_bin"])
    for fld in ("cx", "cy", "r"):
        np.testing.assert_allclose(got[fld], ref[fld], rtol=2e-7, atol=1e-9)


def _end_to_end(det, f, frame):
    ref = O.detect(f.image, f.params)
    got = det.detect(frame, f.params)
    kr, kg = _match(ref, got)
    common = set(kr) & set(kg)
    unmatched = len(set(kr) ^ set(kg))
    for k in common:
        a, b = kr[k], kg[k]
        assert abs(a["cx"] - b["cx"]) <= 0.05 and abs(a["cy"] - b["cy"]) <= 0.05 and abs(a["r"] - b["r"]) <= 0.05
    return ref, got, len(common), unmatched


@pytest.mark.parametrize("name", list(CASES))
def test_end_to_end_rings(det, name):
    say(f"[detect] {name}")
    f = _frame(name)
    ref, got, n_common, unmatched = _end_to_end(det, f, torch.from_numpy(f.image).cuda())
    say(f"  oracle {len(ref)} gpu {len(got)} matched {n_common} unmatched {unmatched}")
    assert unmatched <= max(1, 0.01 * len(ref))


def test_ridge_list_is_a_lossless_representation(det):
    """The ridge list (coordinates and direction codes) stands in for the frame: detection
    from it gives the rings of rd_detect byte for byte, at 12 bytes per ridge (8 as 16-bit
    fields) against 2 bytes per pixel of the u16 frame."""
    say("[ridges] c2 1024x1024: rd_stage_ridges -> rd_detect_ridges vs rd_detect")
    f = synth.config2()
    frame = torch.from_numpy(f.image).cuda()
    xy, q, _ = det.ridges(frame, f.params)
    assert int(xy.max()) < 65536 and int(q.abs().max()) <= 1 << 14
    from_list = det.detect_from_ridges(xy, q, f.width, f.height, f.params)
    direct = det.detect(frame, f.params)
    say(f"  {xy.shape[0]} ridges: {8 * xy.shape[0] / 2**20:.2f} MiB as 16-bit fields vs "
        f"{f.image.nbytes / 2**20:.2f} MiB frame; {len(direct)} rings")
    assert len(direct) > 100 and from_list.tobytes() == direct.tobytes()
    # the order of the list does not matter
    perm = torch.randperm(xy.shape[0], generator=torch.Generator().manual_seed(0)).cuda()
    shuffled = det.detect_from_ridges(xy[perm], q[perm], f.width, f.height, f.params)
    assert shuffled.tobytes() == direct.tobytes()


# ---------------------------------------------------------------- directed edges

def _edge_disc():
    """121 x 121 float32 uniform disc of radius 23.3 around a pixel centre."""
    y, x = np.mgrid[0:121, 0:121].astype(np.float64)
    img = (np.hypot(x - 60, y - 60) < 23.3).astype(np.float32)
    return synth.Frame(img, np.array([60.0]), np.array([60.0]), np.array([23.3]), np.ones(1), np.ones(1),
                       dict(synth.PARAMS_C1, measure=O.MEASURE_EDGE), 0)


def _edge_c1():
    """c1 with directed edges: T at a quarter of the weakest ring's smoothed gradient."""
    f = synth.config1()
    return synth.Frame(f.image, f.cx, f.cy, f.R, f.s, f.A, dict(f.params, measure=O.MEASURE_EDGE, k_threshold=-0.03), 0)


def _edge_ragged():
    """300 x 170 uint16 c2-like frame with directed edges (T = -12 counts / px)."""
    f = synth.config2(seed=21, W=300, H=170, n_rings=12)
    return synth.Frame(f.image, f.cx, f.cy, f.R, f.s, f.A, dict(f.params, measure=O.MEASURE_EDGE, k_threshold=-12.0), 0)


EDGE_CASES = {"disc_121_f32": _edge_disc, "c1_256_f32": _edge_c1, "ragged_300x170_u16": _edge_ragged}


def _check_edge_measure(det, f):
    p = f.params
    m_ref, qx_ref, qy_ref = O.edge_measure(f.image.astype(np.float64), O.f32(p["sigma_smooth"]))
    m, q = det.curvature(torch.from_numpy(f.image).cuda(), p)
    m = m.cpu().numpy().astype(np.float64)
    q = q.cpu().numpy().astype(np.int64)
    err = np.abs(m - m_ref)
    assert np.all(err <= _ktol(m_ref)), float((err / _ktol(m_ref)).max())
    # the direction is undefined where the gradient is within rounding of zero
    defined = -m_ref > 1e-9 * np.abs(f.image).max()
    dqx, dqy = np.abs(q[..., 0] - qx_ref), np.abs(q[..., 1] - qy_ref)
    flips = int((((dqx > 0) | (dqy > 0)) & defined).sum())
    say(f"  |grad| max rel err {float((err / np.maximum(np.abs(m_ref), 1e-300)).max()):.2e}; q flips {flips}")
    assert max(dqx[defined].max(), dqy[defined].max()) <= 1
    assert flips <= max(1, 1e-5 * m.size)


@pytest.mark.parametrize("name", list(EDGE_CASES))
def test_edge_measure_parity(det, name):
    say(f"[edges: measure] {name}")
    _check_edge_measure(det, EDGE_CASES[name]())


@pytest.mark.parametrize("name", list(EDGE_CASES))
def test_edge_sets_and_rings(det, name):
    say(f"[edges: pixels and rings] {name}")
    f = EDGE_CASES[name]()
    ref, got, n = _ridge_sets(det, f)
    sym = set(ref) ^ set(got)
    say(f"  oracle {len(ref)} edge pixels, gpu {len(got)}, mismatched {len(sym)}")
    assert len(ref) > 50 and len(sym) <= max(0, int(1e-4 * len(ref)))
    ring_ref, ring_got, n_common, unmatched = _end_to_end(det, f, torch.from_numpy(f.image).cuda())
    say(f"  rings: oracle {len(ring_ref)} gpu {len(ring_got)} matched {n_common} unmatched {unmatched}")
    assert len(ring_ref) > 0 and unmatched <= max(1, 0.01 * len(ring_ref))


def test_edge_c2_full(det):
    """The headline 1024^2 u16 frame with directed edges, as bench.py times it: measure,
    edge-pixel set and rings against the oracle."""
    say("[edges] c2 1024x1024 u16")
    f = synth.config2()
    f = synth.Frame(f.image, f.cx, f.cy, f.R, f.s, f.A, dict(f.params, measure=O.MEASURE_EDGE, k_threshold=-12.0), 0)
    _check_edge_measure(det, f)
    ref, got, n = _ridge_sets(det, f)
    sym = set(ref) ^ set(got)
    say(f"  oracle {len(ref)} edge pixels, gpu {len(got)}, mismatched {len(sym)}")
    assert len(sym) <= 1e-4 * len(ref)
    ring_ref, ring_got, n_common, unmatched = _end_to_end(det, f, torch.from_numpy(f.image).cuda())
    say(f"  rings: oracle {len(ring_ref)} gpu {len(ring_got)} matched {n_common} unmatched {unmatched}")
    assert unmatched <= max(1, 0.01 * len(ring_ref))


def test_edge_measure_rejected_by_the_differentiable_path(det):
    from paper_1310_1371_amd.native import RdError
    f = _edge_disc()
    with pytest.raises(RdError):
        det.soft_ridges(torch.from_numpy(f.image).cuda(), f.params)


def test_wide_frame_beyond_2048_columns():
    """A 5000 x 48 float32 strip (coordinates past 4095 in the packed 16-bit ridge records),
    with rings along it: accumulator and scores bit-exact from the oracle's ridges, and the
    end-to-end rings within tolerance."""
    from paper_1310_1371_amd.detector import Detector
    say("[wide] 5000 x 48")
    W, H = 5000, 48
    cx = np.array([30.0, 1800.5, 4100.2, 4978.0])
    cy = np.array([24.0, 20.5, 26.0, 23.0])
    R = np.array([14.0, 18.0, 12.5, 16.0])
    s_, A = np.full(4, 1.5), np.ones(4)
    img = synth.render(W, H, np.full((H, W), 0.2), cx, cy, R, s_, A).astype(np.float32)
    f = synth.Frame(img, cx, cy, R, s_, A, dict(synth.PARAMS_C1), 0)
    d = Detector(max_width=W, max_height=64, max_peaks=4096)
    try:
        p = dict(O.DEFAULTS, **f.params)
        xs, ys, qx, qy, xy, q = _oracle_ridge_inputs(f)
        _, A_ref, S_ref = O.detect_from_ridges(xs, ys, qx, qy, W, H, p, return_volumes=True)
        acc, sc = d.accumulate(xy, q, W, H, p)
        np.testing.assert_array_equal(acc.cpu().numpy().astype(np.int64), A_ref)
        np.testing.assert_array_equal(sc.cpu().numpy(), S_ref)
        ref, got, n_common, unmatched = _end_to_end(d, f, torch.from_numpy(f.image).cuda())
        say(f"  oracle {len(ref)} gpu {len(got)} matched {n_common} unmatched {unmatched}")
        assert len(ref) >= 3 and unmatched <= 1
    finally:
        d.close()


def test_end_to_end_c2_full(det):
    say("[detect] c2 1024x1024 u16")
    f = synth.config2()
    ref, got, n_common, unmatched = _end_to_end(det, f, torch.from_numpy(f.image).cuda())
    say(f"  oracle {len(ref)} gpu {len(got)} matched {n_common} unmatched {unmatched}")
    assert unmatched <= max(1, 0.01 * len(ref))
    # sanity against ground truth: most rings are found
    found = sum(1 for j in range(len(f.R))
                if np.min(np.hypot(got["cx"] - f.cx[j], got["cy"] - f.cy[j]) + np.abs(got["r"] - f.R[j])) < 1.5)
    say(f"  truth rings {len(f.R)} found within 1.5 px: {found}")


def test_detect_host_frame_and_repeat_is_bitwise(det):
    say("[detect] host frame, repeated runs")
    f = synth.config1()
    a = det.detect(f.image, f.params)
    b = det.detect(torch.from_numpy(f.image).cuda(), f.params)
    c = det.detect(torch.from_numpy(f.image).cuda(), f.params)
    assert a.tobytes() == b.tobytes() == c.tobytes()


def test_same_storage_different_views(det):
    """Calls alternating between two views that share one base pointer (a full frame and its
    top-left corner, the pitch kept): the context keeps the frame descriptors of the last
    call on the device and uploads new ones only when they differ, so each call must still
    see its own view.  Each result is compared with a fresh context's."""
    from paper_1310_1371_amd.detector import Detector
    say("[detect] alternating views of one buffer")
    f = synth.config2(seed=31, W=512, H=384, n_rings=40)
    full = torch.from_numpy(f.image).cuda()
    part = full[:256, :320]
    with_fresh = []
    for view in (full, part):
        d2 = Detector(max_width=2048, max_height=2048, max_peaks=65536)
        with_fresh.append(d2.detect(view, f.params))
        d2.close()
    assert len(with_fresh[0]) > len(with_fresh[1]) > 0
    for _ in range(2):
        for view, ref in ((full, with_fresh[0]), (part, with_fresh[1]), (full, with_fresh[0])):
            assert det.detect(view, f.params).tobytes() == ref.tobytes()


def test_constant_frame_has_no_rings(det):
    say("[detect] constant frame")
    img = np.full((64, 96), 7.0, np.float32)
    got = det.detect(img, synth.PARAMS_C1)
    assert len(got) == 0
    xy, q, k = det.ridges(img, synth.PARAMS_C1)
    assert xy.shape[0] == 0


def test_single_radius_range(det):
    say("[detect] r_min == r_max")
    f = synth.single_ring(96, 96, 48.0, 47.0, 20.2)
    p = dict(f.params, r_min=20, r_max=20)
    ref = O.detect(f.image, p)
    got = det.detect(f.image, p)
    kr, kg = _match(ref, got)
    assert set(kr) == set(kg)


def test_truncation_reports_required_count(det):
    say("[detect] capacity truncation")
    import ctypes
    from paper_1310_1371_amd import native as N
    from paper_1310_1371_amd.detector import _frame_struct
    f = synth.config1()
    fr = _frame_struct(f.image)
    p = N.make_params(f.params)
    buf = (N.RdRing * 2)()
    n = ctypes.c_int32()
    st = N.lib().rd_detect(det._h, ctypes.byref(fr), ctypes.byref(p), buf, 2, ctypes.byref(n))
    assert st == N.RD_E_TRUNCATED and n.value == len(O.detect(f.image, f.params)) > 2


def test_invalid_arguments_rejected_before_launch(det):
    say("[detect] invalid arguments")
    from paper_1310_1371_amd import native as N
    f = synth.config1()
    with pytest.raises(N.RdError) as e:
        det.detect(f.image, dict(f.params, r_min=0))
    assert e.value.status == N.RD_E_INVALID
    with pytest.raises(N.RdError) as e:
        det.detect(np.zeros((16, 64), np.float32), f.params)
    assert e.value.status == N.RD_E_INVALID
    with pytest.raises(N.RdError) as e:
        det.detect(np.zeros((64, 4096), np.float32), f.params)
    assert e.value.status == N.RD_E_TOO_LARGE
    xy = np.array([[500, 3]], np.int32)
    q = np.array([[16384, 0]], np.int16)
    with pytest.raises(N.RdError) as e:
        det.detect_from_ridges(xy, q, 256, 256, f.params)
    assert e.value.status == N.RD_E_INVALID


@pytest.mark.parametrize("case", ["duplicate", "non_unit", "negative_sign", "zero", "bin_of_257"])
def test_ridge_lists_outside_the_exact_class_are_rejected(det, case):
    """Lists that could break the exactness of the integer votes (a pixel twice, a code that
    is not a unit direction in canonical sign) are refused by both stage entry points, on
    the device, with RD_E_INVALID; the host check agrees."""
    from paper_1310_1371_amd import native as N
    say(f"[ridges] invalid caller list: {case}")
    f = synth.config1()
    xs, ys, qx, qy, xy, q = _oracle_ridge_inputs(f)
    xy, q = xy.copy(), q.copy()
    if case == "duplicate":
        xy = np.concatenate([xy, xy[5:6]])
        q = np.concatenate([q, q[5:6]])
    elif case == "non_unit":
        q[7] = (16384, 200)                  # |q|^2 - 2^28 = 40000 > 2^15
    elif case == "negative_sign":
        q[3] = (-q[3, 0], -q[3, 1]) if q[3, 1] != 0 else (-q[3, 0], 0)
    elif case == "zero":
        q[2] = (0, 0)
    else:                                     # 257 entries in one 16 x 16 bin
        yy, xx = np.mgrid[0:16, 0:16]
        xy = np.concatenate([np.stack([xx.ravel() + 32, yy.ravel() + 32], 1), [[40, 40]]]).astype(np.int32)
        q = np.tile(np.array([[0, 16384]], np.int16), (257, 1))
    assert N.lib().rd_validate_ridges(np.ascontiguousarray(xy, np.int32).ctypes.data,
                                      np.ascontiguousarray(q, np.int16).ctypes.data, len(xy), 256, 256) \
        == N.RD_E_INVALID
    for call in (lambda: det.accumulate(xy, q, 256, 256, f.params, scores=False),
                 lambda: det.detect_from_ridges(xy, q, 256, 256, f.params)):
        with pytest.raises(N.RdError) as e:
            call()
        assert e.value.status == N.RD_E_INVALID
    # the list of step 2 itself passes, and still gives the oracle's rings
    xs, ys, qx, qy, xy, q = _oracle_ridge_inputs(f)
    assert N.lib().rd_validate_ridges(xy.ctypes.data, q.ctypes.data, len(xy), 256, 256) == N.RD_OK
    got = det.detect_from_ridges(xy, q, 256, 256, f.params)
    assert len(got) == len(O.detect_from_ridges(xs, ys, qx, qy, 256, 256, dict(O.DEFAULTS, **f.params)))
