"""Pins of the oracle's classification annulus, fit-rejection rules and integer float
threshold against hand-worked cases (tests/golden/annulus_fit_threshold.txt, each derived in
its comments), exact rational arithmetic and identities of the algebraic circle fit.

Each case sits on a boundary of its rule (a member at exactly (r - w)^2 or (r + w)^2, a
centre that moves exactly w, a score exactly at the threshold), so that moving a bound by one
unit, dropping the clamp of the inner radius, scaling a rejection limit or rounding the
threshold the other way fails at least one of them."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import ridge_hough as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "annulus_fit_threshold.txt")
PI_40 = Fraction("3.141592653589793238462643383279502884197169")


def _cases(key):
    out = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line and line.split("=", 1)[0].strip() == key:
                out.append([int(v) for v in line.split("=", 1)[1].split()])
    return out


def _lattice_circle(R):
    return np.array([(u, v) for u in range(-R, R + 1) for v in range(-R, R + 1) if u * u + v * v == R * R],
                    dtype=np.int64)


# ---------------------------------------------------------------- annulus

def test_annulus_hand_cases():
    cases = _cases("annulus")
    assert len(cases) == 19
    for r, w, u, v, member in cases:
        got = O.annulus_members(np.array([100 + u]), np.array([100 + v]), 100, 100, r, w)
        assert bool(got[0]) == bool(member), (r, w, u, v)


def test_annulus_members_counted_by_the_fit():
    """n_fit of a ring is the number of annulus members (the same hand cases, all at once)."""
    for r, w in ((10, 2), (1, 2), (3, 2)):
        sel = [(u, v, m) for rr, ww, u, v, m in _cases("annulus") if (rr, ww) == (r, w)]
        xs = np.array([50 + u for u, _, _ in sel])
        ys = np.array([60 + v for _, v, _ in sel])
        p = dict(O.DEFAULTS, annulus_halfwidth=w, min_fit_points=3)
        ring = O.fit_rings(xs, ys, [50], [60], [r], [0], p)[0]
        assert ring["n_fit"] == sum(m for _, _, m in sel)


# ---------------------------------------------------------------- fit rejection

def test_fit_rejection_hand_cases():
    pts = _lattice_circle(65)
    assert len(pts) == 36
    a, b = 300, 200
    for dx, dy, r, w, n_fit, ok in _cases("fit"):
        p = dict(O.DEFAULTS, annulus_halfwidth=w, min_fit_points=8)
        ring = O.fit_rings(pts[:, 0] + a + dx, pts[:, 1] + b + dy, [a], [b], [r], [0], p)[0]
        assert ring["n_fit"] == n_fit, (dx, dy, r, w)
        assert ring["fit_ok"] == ok, (dx, dy, r, w)
        if ok:
            assert abs(ring["cx"] - (a + dx)) < 1e-9 and abs(ring["cy"] - (b + dy)) < 1e-9
            assert abs(ring["r"] - 65.0) < 1e-9
        else:        # a rejected fit keeps the Hough peak
            assert (ring["cx"], ring["cy"], ring["r"]) == (float(a), float(b), float(r))


def test_fit_rejects_a_singular_system():
    """Collinear members (v = 0 for all of them) make the normal equations singular: the
    rows of sum v and sum uv, sum v^2 vanish.  The ring keeps its peak."""
    u = np.array([-12, -11, -10, -9, -8, 8, 9, 10, 11, 12])
    p = dict(O.DEFAULTS, annulus_halfwidth=2, min_fit_points=8)
    ring = O.fit_rings(u + 40, np.full(10, 40), [40], [40], [10], [0], p)[0]
    assert ring["n_fit"] == 10 and ring["fit_ok"] == 0
    assert (ring["cx"], ring["cy"], ring["r"]) == (40.0, 40.0, 10.0)


def test_fit_radius_is_the_rms_distance_to_the_fitted_centre():
    """Identity of the algebraic fit: the normal equation of F gives F = -mean(z + D u + E v),
    so r^2 = D^2/4 + E^2/4 - F = mean |p - c|^2 over the members.  The radicand is therefore
    never negative (a negative one could only come from a mistake), and the fitted radius is
    the RMS distance of the members to the fitted centre."""
    rng = np.random.default_rng(7)
    for trial in range(20):
        R = int(rng.integers(12, 40))
        w = int(rng.integers(2, 6))
        n = int(rng.integers(12, 200))
        t = rng.uniform(0, 2 * np.pi, n)
        rad = R + rng.uniform(-w + 0.6, w - 0.6, n)
        xs = np.rint(100 + rng.uniform(-0.4, 0.4) + rad * np.cos(t)).astype(np.int64)
        ys = np.rint(100 + rng.uniform(-0.4, 0.4) + rad * np.sin(t)).astype(np.int64)
        p = dict(O.DEFAULTS, annulus_halfwidth=w, min_fit_points=8)
        ring = O.fit_rings(xs, ys, [100], [100], [R], [0], p)[0]
        if not ring["fit_ok"]:
            continue
        mem = (xs - 100) ** 2 + (ys - 100) ** 2
        keep = (mem >= (R - w) ** 2) & (mem <= (R + w) ** 2)
        rms = np.sqrt(np.mean((xs[keep] - ring["cx"]) ** 2 + (ys[keep] - ring["cy"]) ** 2))
        assert abs(ring["r"] - rms) < 1e-9 * R


# ---------------------------------------------------------------- integer float threshold

def _exact_threshold(f, r):
    """floor(f 2 pi r 2^30) with f the float32 parameter and pi to 42 digits."""
    return math.floor(Fraction(float(np.float32(f))) * 2 * PI_40 * r * 2 ** 30)


def test_score_threshold_hand_values():
    for f1000, r, want in _cases("threshold"):
        p = dict(O.DEFAULTS, peak_fraction=f1000 / 1000.0)
        assert O.score_threshold(r, p) == want


def test_score_threshold_is_the_floor_of_the_exact_product():
    rng = np.random.default_rng(5)
    for _ in range(300):
        f = float(rng.uniform(0.05, 1.5))
        r = int(rng.integers(1, 128))
        want = _exact_threshold(f, r)
        exact = Fraction(float(np.float32(f))) * 2 * PI_40 * r * 2 ** 30
        if exact - want < Fraction(1, 10 ** 4) or want + 1 - exact < Fraction(1, 10 ** 4):
            continue            # within float64 rounding of an integer: no decision to pin
        assert O.score_threshold(r, dict(O.DEFAULTS, peak_fraction=f)) == want


@pytest.mark.parametrize("r", [5, 10, 70])
def test_candidate_needs_a_score_above_f_two_pi(r):
    """A lone voxel is a peak iff S > f 2 pi: S_int = floor(f 2 pi r 2^30) is not (S is at most
    f 2 pi), one unit more is."""
    p = dict(O.DEFAULTS, r_min=r, r_max=r, peak_fraction=0.4)
    thr = _exact_threshold(0.4, r)
    for s_int, is_peak in ((thr, False), (thr + 1, True)):
        S = np.zeros((3, 5, 5), dtype=np.int64)
        S[1, 2, 2] = s_int
        pa, pb, pr, _ = O.peaks(S, r - 1, p)
        assert (len(pa) == 1) == is_peak
        if is_peak:
            assert (pa[0], pb[0], pr[0]) == (2, 2, r)
