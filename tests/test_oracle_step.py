"""Pins of the coarser radius discretisation (SI, "Additional notes": a lower resolution of the
circle parameter space).  Reading: with radius step s the levels are r_min - s + s l,
l = 0 .. floor((r_max - r_min) / s) + 2, peak levels those with radius in [r_min, r_max].

Pinned by hand-listed level radii, brute-force votes at the stepped radii in exact fractions,
an independent peak search over levels of unequal radius with planted cross-level ties, the
reduction to the plain method at s = 1, and single ideal rings whose peak falls on the level
nearest the ridge radius with the circle fit within the plain method's bounds."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import ridge_hough as O
from paper_1310_1371_amd import synth


@pytest.mark.parametrize("r_min,r_max,s,radii", [
    (8, 40, 1, list(range(7, 42))),
    (8, 40, 2, list(range(6, 43, 2))),
    (8, 40, 3, [5, 8, 11, 14, 17, 20, 23, 26, 29, 32, 35, 38, 41]),
    (5, 70, 4, [1, 5, 9, 13, 17, 21, 25, 29, 33, 37, 41, 45, 49, 53, 57, 61, 65, 69, 73]),
    (10, 10, 3, [7, 10, 13]),
])
def test_level_radii_hand_values(r_min, r_max, s, radii):
    got = O.level_radii(dict(O.DEFAULTS, r_min=r_min, r_max=r_max, r_step=s)).tolist()
    assert got == radii


def _brute_votes_at(xs, ys, qx, qy, W, H, radii):
    """Each ridge, each listed radius r and sign: the vote lands at x +/- round-half-up of
    r qx / 2^14 (exact fractions), dropped off the frame."""
    A = np.zeros((len(radii), H, W), dtype=np.int64)
    for l, r in enumerate(radii):
        for x, y, a, b in zip(xs, ys, qx, qy):
            ox = math.floor(Fraction(int(r) * int(a), 16384) + Fraction(1, 2))
            oy = math.floor(Fraction(int(r) * int(b), 16384) + Fraction(1, 2))
            for sg in (1, -1):
                u, v = int(x) + sg * ox, int(y) + sg * oy
                if 0 <= u < W and 0 <= v < H:
                    A[l, v, u] += 1
    return A


def test_votes_at_stepped_radii_match_brute_force():
    rng = np.random.default_rng(17)
    W, H, n = 40, 36, 11
    xs, ys = rng.integers(0, W, n), rng.integers(0, H, n)
    ang = rng.uniform(0, np.pi, n)
    qx, qy = O.direction_code(np.cos(ang), np.sin(ang))
    qx[0], qy[0] = 8192, 14189
    p = dict(O.DEFAULTS, r_min=6, r_max=17, r_step=3)
    radii = O.level_radii(p)
    got = O.vote_radii(xs, ys, qx, qy, W, H, radii)
    np.testing.assert_array_equal(got, _brute_votes_at(xs, ys, qx, qy, W, H, radii.tolist()))


def test_scores_are_per_level_with_the_level_radius():
    """Each level's score is the plain method's score of that radius: the same accumulator
    slice smoothed with the window and weights of the level's own radius."""
    f = synth.config1()
    p3 = dict(O.DEFAULTS, **dict(f.params, r_step=3))
    xs, ys, qx, qy, _ = O.ridges(f.image, p3)
    W = H = 256
    _, A3, S3 = O.detect_from_ridges(xs, ys, qx, qy, W, H, p3, return_volumes=True)
    p1 = dict(p3, r_step=1, r_min=p3["r_min"] - 2)      # plain levels 5 .. 41 cover the stepped ones
    _, A1, S1 = O.detect_from_ridges(xs, ys, qx, qy, W, H, p1, return_volumes=True)
    r1 = O.level_radii(p1).tolist()
    for l, r in enumerate(O.level_radii(p3).tolist()):
        np.testing.assert_array_equal(A3[l], A1[r1.index(r)])
        np.testing.assert_array_equal(S3[l], S1[r1.index(r)])


def _brute_peaks_radii(S, radii, p):
    """Independent: v is a peak iff its level radius lies in [r_min, r_max], S/r > f 2 pi, and
    it beats every voxel of its 3x3x3 box by S/r (exact fractions), ties going to the earlier
    voxel in (level, y, x) order."""
    L, H, W = S.shape
    out = []
    for li in range(L):
        r = int(radii[li])
        if not (p["r_min"] <= r <= p["r_max"]):
            continue
        for y in range(H):
            for x in range(W):
                sv = Fraction(int(S[li, y, x]), r)
                if not sv > Fraction(O.score_threshold(r, p), r):
                    continue
                ok = True
                for lj in range(max(0, li - 1), min(L, li + 2)):
                    for yy in range(max(0, y - 1), min(H, y + 2)):
                        for xx in range(max(0, x - 1), min(W, x + 2)):
                            if (lj, yy, xx) == (li, y, x):
                                continue
                            su = Fraction(int(S[lj, yy, xx]), int(radii[lj]))
                            if su > sv or (su == sv and (lj, yy, xx) < (li, y, x)):
                                ok = False
                if ok:
                    out.append((x, y, r))
    return out


def test_peaks_over_stepped_levels_match_brute_force():
    rng = np.random.default_rng(23)
    p = dict(O.DEFAULTS, r_min=6, r_max=15, r_step=3, peak_fraction=0.05)
    radii = O.level_radii(p)                       # 3, 6, 9, 12, 15, 18
    assert radii.tolist() == [3, 6, 9, 12, 15, 18]
    for trial in range(6):
        S = rng.integers(0, 7, (6, 6, 6)).astype(np.int64) * (2 ** 29) * 3
        S[rng.random(S.shape) < 0.3] = 0
        # cross-level ties in S/r between levels of radius 6 and 9, and 9 and 12
        S[1, 2, 2] = 6 * 2 ** 30
        S[2, 2, 2] = 9 * 2 ** 30
        S[2, 4, 3] = 12 * 2 ** 29
        S[3, 4, 3] = 16 * 2 ** 29
        pa, pb, pr, _ = O.peaks_radii(S, radii, p)
        got = list(zip(pa.tolist(), pb.tolist(), pr.tolist()))
        assert got == _brute_peaks_radii(S, radii, p)


def test_step_one_is_the_plain_method():
    f = synth.config1()
    a = O.detect(f.image, dict(f.params))
    b = O.detect(f.image, dict(f.params, r_step=1))
    assert a.tobytes() == b.tobytes()


@pytest.mark.parametrize("s", [2, 3])
@pytest.mark.parametrize("R", [14.3, 22.7, 33.2])
def test_single_ring_with_a_radius_step(s, R):
    """A single noise-free ring at a pixel centre: one strong peak, at the centre, on a peak
    level within s/2 + 1/2 px of the ridge radius R - v/(2R); the fit (which takes the ridge
    pixels within w = 2 of the level's radius) recovers the centre within 0.05 px and the
    radius within 0.1 px of R - v/(2R), as with the plain method."""
    c = 80
    f = synth.single_ring(161, 161, float(c), float(c), R)
    p = dict(O.DEFAULTS, k_threshold=-0.02, r_min=8, r_max=40, r_step=s)
    rings = O.detect(f.image, p)
    strong = rings[rings["score"] > 3.0]
    assert len(strong) == 1
    ring = strong[0]
    v = 4.0 + 2.0 / 3.0
    r_ridge = R - v / (2 * R)
    assert (ring["a"], ring["b"]) == (c, c)
    assert int(ring["r_bin"]) in O.level_radii(p).tolist()
    assert abs(int(ring["r_bin"]) - r_ridge) <= s / 2 + 0.5
    assert ring["fit_ok"] == 1
    assert abs(ring["cx"] - c) < 0.05 and abs(ring["cy"] - c) < 0.05
    assert abs(ring["r"] - r_ridge) < 0.1
