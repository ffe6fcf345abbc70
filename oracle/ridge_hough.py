"""Plain, slow FP64 CPU oracle of the ridge-directed circle Hough transform.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module; only the
tests, the smoke check and the benchmark's CPU-baseline leg may use it.  It shares no code
with the HIP path: its only common input is the seeded frame generator.

What it computes is the dense, array-based formulation of the method (the "convolution and
array based" version the paper first wrote, Results, "Key algorithmic optimisations"),
which the paper's memory-recycling / hotspot machinery reproduces exactly at lower cost.
All floating point is float64.  Every stage is a function of its own, citing the passage it
follows.  Readings taken where the paper is silent are marked READING at the place they
are taken, with the reason.

Coordinates: x = column, y = row, pixel centres at integers, (0, 0) top-left.
"""
from __future__ import annotations

import math

import numpy as np

Q_ONE = 16384          # fixed-point unit of a direction code component (2^14)
Q_HALF = 8192          # 2^13, rounding offset of the vote shift
W_ONE = 32768          # fixed-point unit of a smoothing weight factor (2^15)
S_SCALE = W_ONE * W_ONE  # 2^30, unit of the integer smoothed score
TAN_PI_8_NUM = 13573   # 13573 / 32768 ~ tan(pi/8): sector boundary of the NMS direction
TAN_PI_8_DEN = 32768
TWO_PI = 6.283185307179586

DEFAULTS = dict(sigma_smooth=2.0, k_threshold=-0.02, r_min=8, r_max=40, vote_threshold=3,
                peak_fraction=0.4, sig_slope=0.05, sig_icpt=0.25, annulus_halfwidth=2,
                min_fit_points=8, measure=0, r_step=1)
MEASURE_RIDGE, MEASURE_EDGE = 0, 1     # directed ridges (Hessian) or directed edges (gradient)


def f32(v) -> float:
    """A parameter as the library receives it: a float32, widened to float64."""
    return float(np.float32(v))


# --------------------------------------------------------------------------------------
# Pre-processing: Gaussian smoothing and 5x5 second-order Sobel derivatives
# (Methods, "Algorithm implementation"; SI, "Detailed algorithm", step 1)
# --------------------------------------------------------------------------------------

def reflect101(idx: np.ndarray, n: int) -> np.ndarray:
    """Border rule READING: mirror about the edge pixel (index -1 -> 1, n -> n-2)."""
    idx = np.abs(np.asarray(idx))
    return np.where(idx > n - 1, 2 * (n - 1) - idx, idx)


def gaussian_taps(sigma: float) -> np.ndarray:
    """Normalised 1D Gaussian, truncated at R = ceil(4 sigma) (READING: 17 taps at sigma 2)."""
    R = int(math.ceil(4.0 * sigma))
    i = np.arange(-R, R + 1, dtype=np.float64)
    g = np.exp(-(i * i) / (2.0 * sigma * sigma))
    return g / g.sum()


def correlate_x(img: np.ndarray, taps) -> np.ndarray:
    """out(y, x) = sum_j taps[j] * img(y, reflect101(x + j - R))."""
    taps = np.asarray(taps, dtype=np.float64)
    R = len(taps) // 2
    W = img.shape[1]
    pad = img[:, reflect101(np.arange(-R, W + R), W)]
    out = np.zeros(img.shape, dtype=np.float64)
    for j, t in enumerate(taps):
        out += t * pad[:, j:j + W]
    return out


def correlate_y(img: np.ndarray, taps) -> np.ndarray:
    """out(y, x) = sum_j taps[j] * img(reflect101(y + j - R), x)."""
    return correlate_x(img.T, taps).T


SOBEL_S5 = (1.0, 4.0, 6.0, 4.0, 1.0)     # smoothing: [1,1]^(*4)
SOBEL_D1 = (-1.0, -2.0, 0.0, 2.0, 1.0)   # first derivative: [1,2,1] * [-1,0,1]
SOBEL_D2 = (1.0, 0.0, -2.0, 0.0, 1.0)    # second derivative: [1,2,1] * [1,-2,1]


def gaussian_smooth(img: np.ndarray, sigma: float) -> np.ndarray:
    g = gaussian_taps(sigma)
    return correlate_y(correlate_x(np.asarray(img, dtype=np.float64), g), g)


def hessian(img: np.ndarray, sigma: float):
    """Ixx, Iyy, Ixy of the smoothed image from 5x5 second-order Sobel kernels divided by
    64, so the result is in image units per px^2 (READING)."""
    G = gaussian_smooth(img, sigma)
    Ixx = correlate_y(correlate_x(G, SOBEL_D2), SOBEL_S5) / 64.0
    Iyy = correlate_y(correlate_x(G, SOBEL_S5), SOBEL_D2) / 64.0
    Ixy = correlate_y(correlate_x(G, SOBEL_D1), SOBEL_D1) / 64.0
    return Ixx, Iyy, Ixy


# --------------------------------------------------------------------------------------
# Principal curvature and direction (Results, "Directed ridge detection & votes
# collection": k_- is the smaller Hessian eigenvalue, X_- its eigenvector)
# --------------------------------------------------------------------------------------

def eigen(Ixx, Iyy, Ixy):
    """Closed-form 2x2 symmetric eigensolve.

    Returns (k_minus, k_plus, xm_x, xm_y) with X_+ = (cos t, sin t), t = atan2(2 Ixy,
    Ixx - Iyy) / 2 and X_- = (-sin t, cos t).  READING: at an isotropic point (the two
    eigenvalues equal) X_- = (0, 1).
    """
    t = 0.5 * (Ixx + Iyy)
    h = 0.5 * (Ixx - Iyy)
    d = np.sqrt(h * h + Ixy * Ixy)
    theta = 0.5 * np.arctan2(2.0 * Ixy, Ixx - Iyy)
    xm_x = -np.sin(theta)
    xm_y = np.cos(theta)
    iso = d == 0.0
    xm_x = np.where(iso, 0.0, xm_x)
    xm_y = np.where(iso, 1.0, xm_y)
    return t - d, t + d, xm_x, xm_y


def direction_code(xm_x, xm_y):
    """READING: X_- as an int16 fixed-point pair q = rint_half_even(2^14 X_-), with the
    sign canonicalised so that qy > 0, or qy == 0 and qx > 0.  Voting then runs in exact
    integer arithmetic."""
    qx = np.rint(Q_ONE * np.asarray(xm_x, dtype=np.float64)).astype(np.int64)
    qy = np.rint(Q_ONE * np.asarray(xm_y, dtype=np.float64)).astype(np.int64)
    neg = (qy < 0) | ((qy == 0) & (qx < 0))
    qx = np.where(neg, -qx, qx)
    qy = np.where(neg, -qy, qy)
    return qx, qy


def curvature(img, sigma):
    """k_- (float64) and the direction code (qx, qy) for every pixel."""
    Ixx, Iyy, Ixy = hessian(img, sigma)
    km, _, xx, xy = eigen(Ixx, Iyy, Ixy)
    qx, qy = direction_code(xx, xy)
    return km, qx, qy


# --------------------------------------------------------------------------------------
# Ridge criterion (Results, "Directed ridge detection": (i) k_- < 0, (ii) k_- a local
# minimum along X_-; SI, "Detailed algorithm", step 2: threshold no greater than zero)
# --------------------------------------------------------------------------------------

def nms_offsets(qx, qy):
    """READING: the neighbour along X_- is the nearest of the 8 lattice directions,
    decided in integers: (1,0) if |qy|/|qx| < 13573/32768 (~tan pi/8), (0,1) if
    |qx|/|qy| < 13573/32768, else (1,1) when qx*qy > 0 and (1,-1) otherwise."""
    ax, ay = np.abs(qx), np.abs(qy)
    horiz = TAN_PI_8_NUM * ax > TAN_PI_8_DEN * ay
    vert = (~horiz) & (TAN_PI_8_NUM * ay > TAN_PI_8_DEN * ax)
    nx = np.where(horiz, 1, np.where(vert, 0, 1))
    ny = np.where(horiz, 0, np.where(vert, 1, np.where(qx * qy > 0, 1, -1)))
    return nx, ny


# --------------------------------------------------------------------------------------
# Directed edges (SI, "Additional notes": the Hessian may be replaced by the gradient; its
# magnitude then takes the place of k_- and must be a local maximum along the gradient)
# --------------------------------------------------------------------------------------

def gradient(img: np.ndarray, sigma: float):
    """Ix, Iy of the smoothed image from 5x5 first-order Sobel kernels (D1 along the
    derivative, S5 across) divided by 128, so the result is in image units per px
    (READING)."""
    G = gaussian_smooth(img, sigma)
    Ix = correlate_y(correlate_x(G, SOBEL_D1), SOBEL_S5) / 128.0
    Iy = correlate_y(correlate_x(G, SOBEL_S5), SOBEL_D1) / 128.0
    return Ix, Iy


def edge_measure(img, sigma):
    """m = -|grad I| (float64) and the direction code of the unit gradient for every
    pixel.  READING: the measure is negated so that the ridge criterion below (m under the
    threshold and a strict minimum along the direction) reads "|grad I| above -T and a
    strict maximum along the gradient"; where the gradient vanishes the direction is
    (0, 1), as at an isotropic Hessian."""
    Ix, Iy = gradient(img, sigma)
    g = np.sqrt(Ix * Ix + Iy * Iy)
    nz = g > 0.0
    safe = np.where(nz, g, 1.0)
    ux = np.where(nz, Ix / safe, 0.0)
    uy = np.where(nz, Iy / safe, 1.0)
    qx, qy = direction_code(ux, uy)
    return -g, qx, qy


def ridge_mask(km, qx, qy, k_threshold):
    """Ridge if k_- < T_k and k_- strictly below both neighbours along X_-.  READING:
    pixels on the 1-px frame border are never ridges."""
    H, W = km.shape
    nx, ny = nms_offsets(qx, qy)
    mask = np.zeros((H, W), dtype=bool)
    ys, xs = np.mgrid[1:H - 1, 1:W - 1]
    dx = nx[1:H - 1, 1:W - 1]
    dy = ny[1:H - 1, 1:W - 1]
    k0 = km[1:H - 1, 1:W - 1]
    kp = km[ys + dy, xs + dx]
    kn = km[ys - dy, xs - dx]
    mask[1:H - 1, 1:W - 1] = (k0 < k_threshold) & (k0 < kp) & (k0 < kn)
    return mask


def ridges(img, params):
    """Ridge list in raster order: (x, y, qx, qy, k) arrays; with measure = 1 the directed
    edges, k then holding -|grad I|."""
    p = dict(DEFAULTS, **params)
    if int(p["measure"]) == MEASURE_EDGE:
        km, qx, qy = edge_measure(np.asarray(img, dtype=np.float64), f32(p["sigma_smooth"]))
    else:
        km, qx, qy = curvature(np.asarray(img, dtype=np.float64), f32(p["sigma_smooth"]))
    m = ridge_mask(km, qx, qy, f32(p["k_threshold"]))
    ys, xs = np.nonzero(m)
    return xs.astype(np.int64), ys.astype(np.int64), qx[ys, xs], qy[ys, xs], km[ys, xs]


# --------------------------------------------------------------------------------------
# Directed voting (Results, "Directed ridge detection": each ridge pixel votes for
# (a, b) = (x, y) +/- r X_- for r in range; one vote adds one; SI, "Additional notes":
# votes over [r_min - 1, r_max + 1], peaks searched in [r_min, r_max])
# --------------------------------------------------------------------------------------

def level_radii(p) -> np.ndarray:
    """Radii of the accumulator levels.  The paper votes over [r_min - 1, r_max + 1] in steps
    of one pixel and searches peaks in [r_min, r_max] (SI, "Additional notes"), and names a
    coarser discretisation of the circle parameter space as a way to trade accuracy for speed
    (same notes).  READING for a radius step s >= 1: the peak levels are r_min, r_min + s,
    ... up to r_max, with one more level a step beyond each end, so level l has radius
    r_min - s + s l, l = 0 .. L - 1, L = floor((r_max - r_min) / s) + 3.  s = 1 is the plain
    method.  READING: the lowest level keeps a radius of at least 1 (r_min - s >= 1), since
    scores at different levels compare as S / r."""
    if int(p["r_min"]) - int(p.get("r_step", 1)) < 1:
        raise ValueError("the lowest level radius r_min - r_step must be at least 1")
    s = int(p.get("r_step", 1))
    L = (int(p["r_max"]) - int(p["r_min"])) // s + 3
    return int(p["r_min"]) - s + s * np.arange(L, dtype=np.int64)


def vote_offset(r, q):
    """READING: rho(r, q) = floor((r q + 2^13) / 2^14), the fixed-point r X_- rounded
    half up."""
    return (np.asarray(r, dtype=np.int64) * np.asarray(q, dtype=np.int64) + Q_HALF) >> 14


def vote(xs, ys, qx, qy, W, H, r_lo, r_hi):
    """Dense integer accumulator A[r - r_lo, b, a] over levels r_lo..r_hi."""
    return vote_radii(xs, ys, qx, qy, W, H, np.arange(r_lo, r_hi + 1))


def vote_radii(xs, ys, qx, qy, W, H, radii):
    """Dense integer accumulator A[l, b, a] at the level radii `radii`.  Votes whose centre
    falls outside the frame are dropped (READING)."""
    L = len(radii)
    A = np.zeros((L, H, W), dtype=np.int64)
    xs = np.asarray(xs, dtype=np.int64)
    ys = np.asarray(ys, dtype=np.int64)
    for li in range(L):
        r = int(radii[li])
        ox = vote_offset(r, qx)
        oy = vote_offset(r, qy)
        for s in (1, -1):
            a = xs + s * ox
            b = ys + s * oy
            ok = (a >= 0) & (a < W) & (b >= 0) & (b < H)
            A[li] += np.bincount(b[ok] * W + a[ok], minlength=H * W).reshape(H, W)
    return A


# --------------------------------------------------------------------------------------
# Radius-dependent smoothing and 1/r normalisation (Results, "Local maxima detection in a
# noisy parameter space"; Methods, "Algorithm implementation": weights
# exp(-((x - x_hotspot)/sigma)^2 / 2) with sigma(r) = 0.05 r + 0.25; SI, "Detailed
# algorithm", step 4: only accumulators exceeding the integer threshold are smoothed)
# --------------------------------------------------------------------------------------

def level_sigma(r, p) -> float:
    """sigma(r) = slope * r + intercept, from the float32 parameters, in float64."""
    return f32(p["sig_slope"]) * r + f32(p["sig_icpt"])


def level_radius(r, p) -> int:
    """Window half-width K(r) = ceil(3 sigma(r)) (READING: truncation at 3 sigma)."""
    return int(math.ceil(3.0 * level_sigma(r, p)))


def weight_factors(r, p) -> np.ndarray:
    """READING: the separable factor exp(-d^2 / (2 sigma^2)), d = 0..K, as 15-bit fixed
    point floor(2^15 e + 1/2), so that the smoothed score and every decision taken on it
    are exact integers."""
    sg = level_sigma(r, p)
    K = level_radius(r, p)
    d = np.arange(K + 1, dtype=np.float64)
    return np.floor(W_ONE * np.exp(-(d * d) / (2.0 * sg * sg)) + 0.5).astype(np.int64)


def score_threshold(r, p) -> int:
    """Integer form of S > f 2 pi at level r: S_int > floor(((f * 2pi) * r) * 2^30)."""
    return int(math.floor(f32(p["peak_fraction"]) * TWO_PI * float(r) * float(S_SCALE)))


def hotspots(A_r, vote_threshold):
    """READING: strict A > T_int ("exceeding")."""
    return A_r > vote_threshold


def smooth_level_int(A_r, hot, r, p):
    """S_int(v) = sum_{|dx|,|dy| <= K} W(|dx|) W(|dy|) A_r(v + d) at hotspots, 0 elsewhere.
    The smoothed, normalised score is S = S_int / (r 2^30).  Outside the frame A = 0."""
    H, W = A_r.shape
    K = level_radius(r, p)
    wf = weight_factors(r, p)
    pad = np.zeros((H + 2 * K, W + 2 * K), dtype=np.int64)
    pad[K:K + H, K:K + W] = A_r
    ys, xs = np.nonzero(hot)
    acc = np.zeros(len(ys), dtype=np.int64)
    for dy in range(-K, K + 1):
        for dx in range(-K, K + 1):
            acc += wf[abs(dx)] * wf[abs(dy)] * pad[ys + K + dy, xs + K + dx]
    out = np.zeros((H, W), dtype=np.int64)
    out[ys, xs] = acc
    return out


def smooth_level_exact(A_r, hot, r, p):
    """The same score with float64 Gaussian weights (no fixed point), divided by r.  Used to
    bound the fixed-point reading, not for decisions."""
    H, W = A_r.shape
    K = level_radius(r, p)
    sg = level_sigma(r, p)
    pad = np.zeros((H + 2 * K, W + 2 * K), dtype=np.float64)
    pad[K:K + H, K:K + W] = A_r
    ys, xs = np.nonzero(hot)
    acc = np.zeros(len(ys), dtype=np.float64)
    for dy in range(-K, K + 1):
        for dx in range(-K, K + 1):
            acc += math.exp(-(dx * dx + dy * dy) / (2.0 * sg * sg)) * pad[ys + K + dy, xs + K + dx]
    out = np.zeros((H, W), dtype=np.float64)
    out[ys, xs] = acc / r
    return out


def smooth(A, r_lo, p):
    """Integer scores for every level of the accumulator (0 off hotspots), levels r_lo, r_lo + 1, ..."""
    return smooth_radii(A, r_lo + np.arange(A.shape[0]), p)


def smooth_radii(A, radii, p):
    """Integer scores for every level (0 off hotspots); level l has radius radii[l] and is
    smoothed within itself with that radius' window."""
    S = np.zeros(A.shape, dtype=np.int64)
    for li in range(A.shape[0]):
        hot = hotspots(A[li], int(p["vote_threshold"]))
        if np.any(hot):
            S[li] = smooth_level_int(A[li], hot, int(radii[li]), p)
    return S


# --------------------------------------------------------------------------------------
# Peak extraction (SI, "Detailed algorithm", step 4: float threshold a fraction of 2 pi,
# then a local maximum by nearest-neighbour comparison in a 3x3x3 voxel box)
# --------------------------------------------------------------------------------------

def peaks(S, r_lo, p):
    """peaks_radii on levels of radius r_lo, r_lo + 1, ..."""
    return peaks_radii(S, r_lo + np.arange(S.shape[0]), p)


def peaks_radii(S, radii, p):
    """Candidates: level radius r in [r_min, r_max], S > f 2 pi.  A candidate v is a peak if
    S(v) >= S(u) for all 26 neighbours u in the volume (the adjacent levels, whatever their
    radii) and S(v) > S(u) for those u before v in (level, y, x) order (READING: the
    tie-break keeps a plateau's first voxel).  Scores at different levels compare as
    S_int / r, done exactly by cross-multiplication with the levels' radii.
    Returns int64 arrays (a, b, r, S_int) in ascending (r, b, a)."""
    L, H, W = S.shape
    r_min, r_max = int(p["r_min"]), int(p["r_max"])
    out = []
    for li in range(L):
        r = int(radii[li])
        if r < r_min or r > r_max:
            continue
        thr = score_threshold(r, p)
        ys, xs = np.nonzero(S[li] > thr)
        for y, x in zip(ys.tolist(), xs.tolist()):
            sv = int(S[li, y, x])
            is_peak = True
            for dl in (-1, 0, 1):
                lj = li + dl
                if lj < 0 or lj >= L:
                    continue
                ru = int(radii[lj])
                for dy in (-1, 0, 1):
                    yy = y + dy
                    if yy < 0 or yy >= H:
                        continue
                    for dx in (-1, 0, 1):
                        xx = x + dx
                        if (dl, dy, dx) == (0, 0, 0) or xx < 0 or xx >= W:
                            continue
                        su = int(S[lj, yy, xx])
                        lhs, rhs = sv * ru, su * r
                        earlier = (dl, dy, dx) < (0, 0, 0)
                        if (earlier and not lhs > rhs) or ((not earlier) and not lhs >= rhs):
                            is_peak = False
                            break
                    if not is_peak:
                        break
                if not is_peak:
                    break
            if is_peak:
                out.append((x, y, r, sv))
    if not out:
        z = np.zeros(0, dtype=np.int64)
        return z, z, z, z
    arr = np.array(out, dtype=np.int64)
    return arr[:, 0], arr[:, 1], arr[:, 2], arr[:, 3]


# --------------------------------------------------------------------------------------
# Classification and sub-pixel circle fit (Results, "Ridge points classification &
# sub-pixel accuracy"; SI, "Detailed algorithm", step 5)
# --------------------------------------------------------------------------------------

def annulus_members(xs, ys, a, b, r, w):
    """READING: ridge pixels with (max(r - w, 0))^2 <= (x-a)^2 + (y-b)^2 <= (r + w)^2,
    decided in integers; non-exclusive between peaks."""
    u = xs - a
    v = ys - b
    z = u * u + v * v
    lo = max(r - w, 0)
    return (z >= lo * lo) & (z <= (r + w) * (r + w))


def kasa_moments(u, v):
    """Exact integer normal-equation moments of the algebraic circle fit."""
    z = u * u + v * v
    return dict(n=len(u), su=int(u.sum()), sv=int(v.sum()), suu=int((u * u).sum()),
                suv=int((u * v).sum()), svv=int((v * v).sum()), sz=int(z.sum()),
                suz=int((u * z).sum()), svz=int((v * z).sum()))


def kasa_fit(m):
    """READING (the paper names no fit): the Kasa algebraic fit, minimising
    sum (z + D u + E v + F)^2 in peak-centred coordinates; solved in float64.
    Returns (D, E, F) or None if the system is singular."""
    M = np.array([[m["suu"], m["suv"], m["su"]],
                  [m["suv"], m["svv"], m["sv"]],
                  [m["su"], m["sv"], m["n"]]], dtype=np.float64)
    rhs = -np.array([m["suz"], m["svz"], m["sz"]], dtype=np.float64)
    try:
        D, E, F = np.linalg.solve(M, rhs)
    except np.linalg.LinAlgError:
        return None
    return D, E, F


RING_DTYPE = np.dtype([("cx", np.float64), ("cy", np.float64), ("r", np.float64),
                       ("score", np.float64), ("a", np.int64), ("b", np.int64),
                       ("r_bin", np.int64), ("n_fit", np.int64), ("fit_ok", np.int64)])


def fit_rings(xs, ys, pa, pb, pr, pS, p):
    """One ring per peak.  READING: the fit is rejected (fit_ok = 0, the ring keeps the
    integer peak) if fewer than min_fit_points members, the system is singular or not
    finite, the centre moves more than w from (a, b) or the radius more than w from r."""
    w = int(p["annulus_halfwidth"])
    nmin = int(p["min_fit_points"])
    xs = np.asarray(xs, dtype=np.int64)
    ys = np.asarray(ys, dtype=np.int64)
    out = np.zeros(len(pa), dtype=RING_DTYPE)
    for j in range(len(pa)):
        a, b, r, s_int = int(pa[j]), int(pb[j]), int(pr[j]), int(pS[j])
        mem = annulus_members(xs, ys, a, b, r, w)
        m = kasa_moments(xs[mem] - a, ys[mem] - b)
        cx, cy, rr, ok = float(a), float(b), float(r), 0
        if m["n"] >= nmin:
            sol = kasa_fit(m)
            if sol is not None:
                D, E, F = sol
                ccx, ccy = a - D / 2.0, b - E / 2.0
                r2 = D * D / 4.0 + E * E / 4.0 - F
                if np.isfinite(ccx) and np.isfinite(ccy) and np.isfinite(r2) and r2 >= 0:
                    rf = math.sqrt(r2)
                    if math.hypot(ccx - a, ccy - b) <= w and abs(rf - r) <= w:
                        cx, cy, rr, ok = ccx, ccy, rf, 1
        out[j] = (cx, cy, rr, s_int / (r * float(S_SCALE)), a, b, r, m["n"], ok)
    return out


# --------------------------------------------------------------------------------------
# The whole plain pipeline
# --------------------------------------------------------------------------------------

def detect_from_ridges(xs, ys, qx, qy, W, H, params, return_volumes=False):
    p = dict(DEFAULTS, **params)
    radii = level_radii(p)
    A = vote_radii(xs, ys, qx, qy, W, H, radii)
    S = smooth_radii(A, radii, p)
    pa, pb, pr, pS = peaks_radii(S, radii, p)
    rings = fit_rings(xs, ys, pa, pb, pr, pS, p)
    if return_volumes:
        return rings, A, S
    return rings


def detect(img, params, return_all=False):
    """Frame -> ring list (RING_DTYPE, ascending (r_bin, b, a))."""
    p = dict(DEFAULTS, **params)
    img = np.asarray(img)
    H, W = img.shape
    xs, ys, qx, qy, k = ridges(img, p)
    if return_all:
        rings, A, S = detect_from_ridges(xs, ys, qx, qy, W, H, p, return_volumes=True)
        return rings, dict(xs=xs, ys=ys, qx=qx, qy=qy, k=k, A=A, S=S)
    return detect_from_ridges(xs, ys, qx, qy, W, H, p)
