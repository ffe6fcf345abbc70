"""Pins of the FP64 oracle against closed forms, library routines, hand values and brute
force.  None of these re-types the oracle's own formula: each check comes from the
mathematics or from an independent formulation, chosen so that a dropped term, a wrong sign
or index or a transposed operand fails at least one of them."""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import ridge_hough as O
from paper_1310_1371_amd import synth

GOLDEN = __file__.replace("test_oracle_pins.py", "golden/hand_values.txt")


def _golden():
    out = {}
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                key, val = line.split("=", 1)
                out[key.strip()] = [int(v) for v in val.split()]
    return out


# ---------------------------------------------------------------- borders and kernels

def test_reflect101_hand_table():
    g = _golden()
    got = O.reflect101(np.arange(-3, 8), 5).tolist()
    assert got == g["reflect101_n5_from_-3_to_7"]


def test_gaussian_taps_shape():
    g = O.gaussian_taps(2.0)
    assert len(g) == 17
    assert abs(g.sum() - 1.0) < 1e-15
    i = np.arange(-8, 9)
    np.testing.assert_allclose(g / g[8], np.exp(-(i * i) / 8.0), rtol=1e-15)


def test_hessian_exact_on_quadratics():
    """Gaussian smoothing adds only a constant to a quadratic and the 5x5 second-order
    Sobel kernels are exact on polynomials of degree 2: Ixx = 2a, Ixy = b, Iyy = 2c away
    from the border."""
    H, W = 48, 64
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    a, b, c, d, e, f = 0.013, -0.021, 0.007, 0.5, -0.3, 11.0
    img = a * x * x + b * x * y + c * y * y + d * x + e * y + f
    Ixx, Iyy, Ixy = O.hessian(img, 2.0)
    inner = (slice(11, H - 11), slice(11, W - 11))
    np.testing.assert_allclose(Ixx[inner], 2 * a, atol=1e-12)
    np.testing.assert_allclose(Iyy[inner], 2 * c, atol=1e-12)
    np.testing.assert_allclose(Ixy[inner], b, atol=1e-12)


def _full_kernel(ky, kx, sigma):
    g = O.gaussian_taps(sigma)
    return np.outer(np.convolve(g, ky), np.convolve(g, kx))


def test_hessian_equals_full_2d_kernel_with_mirror_border():
    """The two-step separable computation equals one 2D correlation of the raw image with
    the composite (Gaussian * Sobel) kernel under scipy's 'mirror' border (= reflect-101),
    everywhere including the border."""
    rng = np.random.default_rng(5)
    img = rng.normal(0, 1, (37, 41)) * 100 + 500
    Ixx, Iyy, Ixy = O.hessian(img, 2.0)
    S5 = [1, 4, 6, 4, 1]
    D1 = [-1, -2, 0, 2, 1]
    D2 = [1, 0, -2, 0, 1]
    for got, ky, kx in ((Ixx, S5, D2), (Iyy, D2, S5), (Ixy, D1, D1)):
        ref = ndi.correlate(img, _full_kernel(ky, kx, 2.0) / 64.0, mode="mirror")
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-10)


# ---------------------------------------------------------------- directed-edge gradient

def test_gradient_exact_on_linear_ramps():
    """On I = a x + b y + c the normalised Gaussian keeps the ramp and the first-order Sobel
    pair divided by 128 returns (a, b) exactly, away from the mirrored border."""
    y, x = np.mgrid[0:64, 0:72].astype(np.float64)
    for a, b in ((0.7, -0.3), (-2.5, 0.0), (0.0, 1.25)):
        Ix, Iy = O.gradient(a * x + b * y + 5.0, 2.0)
        np.testing.assert_allclose(Ix[12:-12, 12:-12], a, rtol=0, atol=1e-12)
        np.testing.assert_allclose(Iy[12:-12, 12:-12], b, rtol=0, atol=1e-12)


def test_gradient_equals_full_2d_kernel_with_mirror_border():
    """The separable gradient equals one 2D correlation of the raw image with the composite
    (Gaussian * Sobel) kernel under scipy's 'mirror' border (= reflect-101)."""
    rng = np.random.default_rng(7)
    img = rng.normal(0, 1, (37, 41)) * 100 + 500
    Ix, Iy = O.gradient(img, 2.0)
    S5 = [1, 4, 6, 4, 1]
    D1 = [-1, -2, 0, 2, 1]
    for got, ky, kx in ((Ix, S5, D1), (Iy, D1, S5)):
        ref = ndi.correlate(img, _full_kernel(ky, kx, 2.0) / 128.0, mode="mirror")
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-10)


def _disc(W, H, cx, cy, R):
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    return (np.hypot(x - cx, y - cy) < R).astype(np.float64)


def test_edge_measure_of_a_disc():
    """A uniform disc: -|grad I| is strongest on the rim (the measure's minimum along the
    row through the centre lies within one pixel of x = c +/- R), and each edge pixel's code
    is the radial direction (the unit gradient points at the centre, up to the sign the code
    canonicalises)."""
    c, R = 60, 23.3
    img = _disc(121, 121, c, c, R)
    m, qx, qy = O.edge_measure(img, 2.0)
    row = m[c]
    assert abs(int(np.argmin(row[:c])) - (c - R)) <= 1.0
    assert abs(int(c + np.argmin(row[c:])) - (c + R)) <= 1.0
    xs, ys, eqx, eqy, k = O.ridges(img, dict(O.DEFAULTS, measure=O.MEASURE_EDGE, k_threshold=-0.02))
    assert len(xs) > 100
    d = np.hypot(xs - c, ys - c)
    assert np.all(np.abs(d - R) < 1.5)
    cos = np.abs(eqx * (xs - c) + eqy * (ys - c)) / (O.Q_ONE * d)
    assert cos.min() > 0.99


def test_edge_mode_finds_a_disc_at_its_centre_and_radius():
    """With directed edges a uniform disc of radius R gives its strongest ring at the disc's
    centre, and the Kasa fit of its rim lands within 0.05 px of the centre and 0.3 px of R
    (a blurred disc's steepest point moves outward by about sigma^2 / 2R)."""
    c, R = 60, 23.3
    img = _disc(121, 121, c, c, R)
    p = dict(O.DEFAULTS, measure=O.MEASURE_EDGE, k_threshold=-0.02, r_min=8, r_max=40)
    rings = O.detect(img, p)
    top = rings[np.argmax(rings["score"])]
    assert (top["a"], top["b"]) == (c, c)
    assert top["fit_ok"] == 1
    assert abs(top["cx"] - c) < 0.05 and abs(top["cy"] - c) < 0.05
    assert abs(top["r"] - R) < 0.3


# ---------------------------------------------------------------- eigensolve

def test_eigen_matches_numpy_eigh():
    rng = np.random.default_rng(1)
    n = 100_000
    Ixx, Iyy, Ixy = rng.normal(0, 1, (3, n))
    Ixx[:10] = Iyy[:10]          # some near-degenerate cases
    km, kp, xx, xy = O.eigen(Ixx, Iyy, Ixy)
    M = np.stack([np.stack([Ixx, Ixy], -1), np.stack([Ixy, Iyy], -1)], -2)
    w, v = np.linalg.eigh(M)
    scale = np.maximum(np.abs(w).max(axis=1), 1e-300)
    np.testing.assert_array_less(np.abs(km - w[:, 0]) / scale, 1e-13)
    np.testing.assert_array_less(np.abs(kp - w[:, 1]) / scale, 1e-13)
    gap = w[:, 1] - w[:, 0]
    ok = gap > 1e-6 * scale
    cross = np.abs(xx * v[:, 1, 0] - xy * v[:, 0, 0])       # |sin angle| between them
    assert np.all(cross[ok] < 1e-11)
    np.testing.assert_allclose(np.hypot(xx, xy), 1.0, rtol=1e-14)


def test_eigen_closed_forms():
    g = _golden()
    # diagonal: smaller eigenvalue along the axis that has it
    km, kp, xx, xy = O.eigen(np.array([-3.0, 2.0]), np.array([1.0, -5.0]), np.array([0.0, 0.0]))
    assert km.tolist() == [-3.0, -5.0] and kp.tolist() == [1.0, 2.0]
    qx, qy = O.direction_code(xx, xy)
    assert list(zip(qx.tolist(), qy.tolist())) == [(16384, 0), (0, 16384)]
    # isotropic point -> (0, 1) by the stated reading
    km, kp, xx, xy = O.eigen(np.array([2.0]), np.array([2.0]), np.array([0.0]))
    assert (km[0], kp[0], xx[0], xy[0]) == (2.0, 2.0, 0.0, 1.0)
    # pure shear [[0, b], [b, 0]]: eigenvalues -|b|, |b|, eigenvectors at 45 degrees
    for b, key in ((1.5, "q_shear_b_pos"), (-1.5, "q_shear_b_neg")):
        km, kp, xx, xy = O.eigen(np.array([0.0]), np.array([0.0]), np.array([b]))
        assert abs(km[0] + 1.5) < 1e-15 and abs(kp[0] - 1.5) < 1e-15
        qx, qy = O.direction_code(xx, xy)
        assert [int(qx[0]), int(qy[0])] == g[key]


def test_gaussian_ring_curvature_closed_form():
    """I = A exp(-(rho - R)^2 / 2 s^2): on the crest the radial curvature after smoothing
    is about -A s / s_eff^3 with s_eff^2 = s^2 + sigma_s^2 + 2/3 (the Sobel pair adds
    variance 1/2 + 1/6 along its axis), and X_- points along the radius."""
    for R in (20.0, 30.0, 45.0):
        c = 100.0
        f = synth.single_ring(201, 201, c, c, R, s=1.5, A=1.0)
        km, qx, qy = O.curvature(f.image.astype(np.float64), 2.0)
        s_eff = math.sqrt(1.5 ** 2 + 4.0 + 2.0 / 3.0)
        want = -1.5 / s_eff ** 3
        for (y, x, rad) in ((100, 100 + int(R), (1, 0)), (100 - int(R), 100, (0, 1))):
            assert abs(km[y, x] / want - 1.0) < 0.05
            ang = math.atan2(abs(qx[y, x] * rad[1] - qy[y, x] * rad[0]),
                             abs(qx[y, x] * rad[0] + qy[y, x] * rad[1]))
            assert ang < 1e-2


# ---------------------------------------------------------------- direction code and votes

def test_direction_code_and_vote_offset_hand_values():
    g = _golden()
    qx, qy = O.direction_code(np.array([1.0, math.sqrt(0.5), -1.0, 0.0]),
                              np.array([0.0, math.sqrt(0.5), 0.0, -1.0]))
    assert [int(v) for v in qx] == g["q_axis_45_neg_x_neg_y"][0::2]
    assert [int(v) for v in qy] == g["q_axis_45_neg_x_neg_y"][1::2]
    assert int(O.vote_offset(10, 11585)) == g["rho_r10_q11585"][0]
    assert int(O.vote_offset(10, 16384)) == 10
    # exact halves round up: +0.5 -> 1, -0.5 -> 0, -1.5 -> -1
    assert O.vote_offset(1, 8192) == 1 and O.vote_offset(1, -8192) == 0
    assert O.vote_offset(3, -8192) == -1


def _brute_votes(xs, ys, qx, qy, W, H, r_lo, r_hi):
    A = np.zeros((r_hi - r_lo + 1, H, W), dtype=np.int64)
    for x, y, a, b in zip(xs, ys, qx, qy):
        for r in range(r_lo, r_hi + 1):
            ox = math.floor(Fraction(r * int(a), 16384) + Fraction(1, 2))
            oy = math.floor(Fraction(r * int(b), 16384) + Fraction(1, 2))
            for s in (1, -1):
                cx, cy = int(x) + s * ox, int(y) + s * oy
                if 0 <= cx < W and 0 <= cy < H:
                    A[r - r_lo, cy, cx] += 1
    return A


def test_counter_bound_at_the_largest_radius():
    """A counter at level r receives at most one vote per lattice offset rho(r, q) (a pixel
    votes once per sign, and its two signs cannot meet at r >= 1), so the number of distinct
    offsets over every direction code bounds every count.  At r = 127 (r_max <= 126, plus the
    neighbour level) it stays far below 4096: two 8-tap bands of smoothing weights <= 2^15
    then sum below 2^31, which the fused kernel relies on."""
    th = np.linspace(0.0, 2.0 * np.pi, 400_000, endpoint=False)
    qx, qy = O.direction_code(np.cos(th), np.sin(th))
    codes = np.unique(np.stack([qx, qy], 1), axis=0)
    offs = set()
    for sgn in (1, -1):
        ox = O.vote_offset(127, sgn * codes[:, 0])
        oy = O.vote_offset(127, sgn * codes[:, 1])
        offs.update(zip(ox.tolist(), oy.tolist()))
    n = len(offs)
    assert 2 * np.pi * 127 < n < 1600
    assert 16 * n * 2 ** 15 < 2 ** 31


def test_vote_matches_brute_force():
    rng = np.random.default_rng(7)
    W, H = 24, 20
    n = 9
    xs = rng.integers(0, W, n)
    ys = rng.integers(0, H, n)
    ang = rng.uniform(0, np.pi, n)
    qx, qy = O.direction_code(np.cos(ang), np.sin(ang))
    qx[0], qy[0] = 8192, 14189       # half-way cases
    got = O.vote(xs, ys, qx, qy, W, H, 2, 11)
    np.testing.assert_array_equal(got, _brute_votes(xs, ys, qx, qy, W, H, 2, 11))


# ---------------------------------------------------------------- ridge criterion

def _nearest_sector(phi):
    dirs = [(1, 0), (1, 1), (0, 1), (-1, 1)]
    best = max(dirs, key=lambda d: abs(math.cos(phi) * d[0] + math.sin(phi) * d[1]) / math.hypot(*d))
    return best


@pytest.mark.parametrize("deg", [0, 10, 35, 45, 55, 80, 90, 100, 125, 135, 150, 170])
def test_straight_ridge_is_the_nearest_pixel_line(deg):
    """For I = f(n.p - c) every discrete Hessian is a function of delta_p = n.p - c, even
    in delta, so with the neighbour step Delta = |n . d_sector| the ridge set is exactly
    {p : |delta_p| < Delta / 2}."""
    phi = math.radians(deg)
    n = (math.cos(phi), math.sin(phi))
    H = W = 72
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    rng = np.random.default_rng(deg)
    d = _nearest_sector(phi)
    Delta = abs(n[0] * d[0] + n[1] * d[1])
    for _ in range(20):
        c = n[0] * 36 + n[1] * 36 + rng.uniform(-0.5, 0.5)
        delta = n[0] * x + n[1] * y - c
        margin = np.abs(np.abs(delta) - Delta / 2)
        if margin[12:-12, 12:-12].min() > 0.02:
            break
    img = np.exp(-(delta ** 2) / (2 * 1.5 ** 2))
    km, qx, qy = O.curvature(img, 2.0)
    mask = O.ridge_mask(km, qx, qy, -0.01)
    want = np.abs(delta) < Delta / 2
    inner = (slice(12, H - 12), slice(12, W - 12))
    np.testing.assert_array_equal(mask[inner], want[inner])
    assert want[inner].sum() > 20


# ---------------------------------------------------------------- smoothing

def test_sigma_and_window_radius():
    p = O.DEFAULTS
    assert abs(O.level_sigma(40, p) - 2.25) < 1e-6
    assert [O.level_radius(r, p) for r in (8, 40, 70)] == [2, 7, 12]
    wf = O.weight_factors(40, p)
    assert wf[0] == 32768
    np.testing.assert_allclose(wf / 32768.0, np.exp(-np.arange(8) ** 2 / (2 * 2.25 ** 2)),
                               atol=2 ** -16 + 1e-7)


def test_smoothing_impulse_closed_form():
    """A hotspot next to an impulse: S(v) = (A(v) + n exp(-|d|^2 / 2 sigma^2)) / r."""
    p = dict(O.DEFAULTS)
    r = 30
    sg = O.level_sigma(r, p)
    for d in ((0, 0), (1, 0), (0, 2), (-3, 1), (4, -4)):
        A = np.zeros((40, 40), dtype=np.int64)
        A[20, 20] = 4
        if d != (0, 0):
            A[20 + d[1], 20 + d[0]] = 100
        hot = np.zeros_like(A, dtype=bool)
        hot[20, 20] = True
        S = O.smooth_level_int(A, hot, r, p)
        want = (4 + (100 * math.exp(-(d[0] ** 2 + d[1] ** 2) / (2 * sg * sg)) if d != (0, 0) else 0)) / r
        got = S[20, 20] / (r * 2.0 ** 30)
        assert abs(got - want) < 100 * 2 ** -15 / r
        assert S[hot == False].max() == 0  # noqa: E712


def test_hotspot_threshold_is_strict():
    """Only accumulators exceeding the integer threshold are hotspots."""
    A = np.array([[2, 3, 4]], dtype=np.int64)
    assert O.hotspots(A, 3).tolist() == [[False, False, True]]


def test_smoothing_fixed_point_within_bound_of_exact_weights():
    rng = np.random.default_rng(3)
    p = dict(O.DEFAULTS)
    for r in (7, 20, 41):
        A = rng.poisson(2.0, (50, 60)).astype(np.int64)
        hot = O.hotspots(A, 3)
        Si = O.smooth_level_int(A, hot, r, p) / (r * 2.0 ** 30)
        Se = O.smooth_level_exact(A, hot, r, p)
        K = O.level_radius(r, p)
        box = ndi.uniform_filter(A.astype(np.float64), 2 * K + 1, mode="constant") * (2 * K + 1) ** 2
        assert np.all(np.abs(Si - Se) <= box * 2 ** -15 / r + 1e-12)


def test_ideal_ring_score_bound():
    """With unnormalised weights (peak weight 1) S at the apex is at most (#ridge pixels)/r,
    each ridge pixel giving at most one vote inside one window; an ideal ring brings about
    one vote per unit of perimeter to its centre, so S is of order 2 pi.  (On a square
    lattice a diagonal crest yields up to sqrt(2) ridge pixels per unit length, so the count
    lies between 4 sqrt(2) R and 2 sqrt(2) pi R.)"""
    f = synth.single_ring(161, 161, 80.0, 80.0, 30.3)
    p = dict(O.DEFAULTS, k_threshold=-0.02)
    rings, d = O.detect(f.image, p, return_all=True)
    n_ridge = len(d["xs"])
    assert len(rings) >= 1
    top = rings[np.argmax(rings["score"])]
    assert top["score"] <= n_ridge / top["r_bin"] + 1e-9
    R = 30.3
    assert 4 * math.sqrt(2) * R <= n_ridge <= 2 * math.sqrt(2) * math.pi * R
    assert 0.7 * 2 * math.pi < top["score"]


# ---------------------------------------------------------------- peak extraction

def _brute_peaks(S, r_lo, p):
    """Independent formulation: v is a peak iff it is a candidate and, ordering voxels by
    (S/r exactly, then earlier-first), it beats every voxel of its 3x3x3 box."""
    L, H, W = S.shape
    out = []
    for li in range(L):
        r = r_lo + li
        if not (p["r_min"] <= r <= p["r_max"]):
            continue
        for y in range(H):
            for x in range(W):
                sv = Fraction(int(S[li, y, x]), r)
                if not float(sv) / 2 ** 30 > p["peak_fraction"] * 2 * math.pi:
                    continue
                ok = True
                for lj in range(max(0, li - 1), min(L, li + 2)):
                    for yy in range(max(0, y - 1), min(H, y + 2)):
                        for xx in range(max(0, x - 1), min(W, x + 2)):
                            if (lj, yy, xx) == (li, y, x):
                                continue
                            su = Fraction(int(S[lj, yy, xx]), r_lo + lj)
                            if su > sv or (su == sv and (lj, yy, xx) < (li, y, x)):
                                ok = False
                if ok:
                    out.append((x, y, r))
    return out


def test_peaks_match_brute_force_with_planted_ties():
    rng = np.random.default_rng(11)
    p = dict(O.DEFAULTS, r_min=3, r_max=6, peak_fraction=0.05)
    for trial in range(6):
        S = rng.integers(0, 6, (6, 6, 6)).astype(np.int64) * (2 ** 29)
        S[rng.random(S.shape) < 0.3] = 0
        # plant plateaus: equal scores at the same level and equal S/r across levels
        S[2, 1, 1] = S[2, 1, 2] = 9 * 2 ** 29
        S[2, 4, 4] = 4 * 2 ** 29            # level r = 4: S/r = 2^29
        S[3, 4, 4] = 5 * 2 ** 29            # level r = 5: the same S/r, a cross-level tie
        pa, pb, pr, _ = O.peaks(S, 2, p)
        got = list(zip(pa.tolist(), pb.tolist(), pr.tolist()))
        assert got == _brute_peaks(S, 2, p)


# ---------------------------------------------------------------- circle fit

def _lattice_circle(R):
    pts = [(u, v) for u in range(-R, R + 1) for v in range(-R, R + 1) if u * u + v * v == R * R]
    return np.array(pts, dtype=np.int64)


def test_fit_exact_on_lattice_circles():
    """Integer points exactly on a circle give the circle back exactly, also when the
    Hough peak is one pixel off the centre."""
    p = dict(O.DEFAULTS, min_fit_points=8)
    for R, (a, b) in ((25, (50, 60)), (65, (100, 90)), (5, (20, 20))):
        pts = _lattice_circle(R)
        xs, ys = pts[:, 0] + a, pts[:, 1] + b
        for da, db in ((0, 0), (1, 0), (0, -1)):
            rings = O.fit_rings(xs, ys, [a + da], [b + db], [R], [0], p)
            assert rings["fit_ok"][0] == 1
            assert abs(rings["cx"][0] - a) < 1e-12 and abs(rings["cy"][0] - b) < 1e-12
            assert abs(rings["r"][0] - R) < 1e-12


def test_fit_rejects_too_few_points():
    p = dict(O.DEFAULTS, min_fit_points=8)
    pts = _lattice_circle(5)[:7]
    rings = O.fit_rings(pts[:, 0] + 10, pts[:, 1] + 10, [10], [10], [5], [0], p)
    assert rings["fit_ok"][0] == 0 and rings["cx"][0] == 10.0 and rings["n_fit"][0] == 7


# ---------------------------------------------------------------- end to end

@pytest.mark.parametrize("R", [14.3, 22.7, 33.2])
def test_single_ring_invariant(R):
    """A single noise-free ring at a pixel centre gives one peak at that centre; the fitted
    centre is within 0.05 px and the radius within 0.1 px of R - v/(2R), v = sigma_s^2 +
    2/3 being the blur variance added to the ring (first-order inward shift of the ridge
    of a blurred ring)."""
    c = 80
    f = synth.single_ring(161, 161, float(c), float(c), R)
    p = dict(O.DEFAULTS, k_threshold=-0.02, r_min=8, r_max=40)
    rings = O.detect(f.image, p)
    strong = rings[rings["score"] > 3.0]
    assert len(strong) == 1
    ring = strong[0]
    assert (ring["a"], ring["b"]) == (c, c)
    v = 4.0 + 2.0 / 3.0
    assert ring["fit_ok"] == 1
    assert abs(ring["cx"] - c) < 0.05 and abs(ring["cy"] - c) < 0.05
    assert abs(ring["r"] - (R - v / (2 * R))) < 0.1


def test_config1_rings_found():
    f = synth.config1()
    rings = O.detect(f.image, f.params)
    # every ring whose centre is at least R from two borders is found within 0.5 px
    found = 0
    for j in range(len(f.R)):
        d = np.hypot(rings["cx"] - f.cx[j], rings["cy"] - f.cy[j])
        if d.min() < 0.5 and abs(rings["r"][np.argmin(d)] - f.R[j]) < 0.5:
            found += 1
    assert found >= 7
