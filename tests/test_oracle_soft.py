"""Pins of the FP64 differentiable-path oracle: adjoint identities, brute-force splats, closed
forms of the ring-profile fit, central finite differences at step 1e-6 and convergence of the
refinement on a noise-free ring."""
import math

import numpy as np
import pytest

from oracle import ridge_hough as O
from oracle import soft as S
from paper_1310_1371_amd import synth

EPS = np.finfo(np.float64).eps
H_FD = 1e-6
RTOL_FD = 1e-4


# ---------------------------------------------------------------- Hessian adjoint

def test_correlate_adjoint_hand_value():
    # W = 5, taps (1, 2, 3): out(0) = 1 in(reflect(-1) = 1) + 2 in(0) + 3 in(1), so the
    # transpose of the unit impulse at x = 0 puts 2 at q = 0 and 1 + 3 at q = 1
    d = np.zeros((1, 5))
    d[0, 0] = 1.0
    assert S.correlate_x_adjoint(d, (1.0, 2.0, 3.0)).tolist() == [[2.0, 4.0, 0.0, 0.0, 0.0]]
    d = np.zeros((1, 5))
    d[0, 4] = 1.0          # out(4) = 1 in(3) + 2 in(4) + 3 in(reflect(5) = 3)
    assert S.correlate_x_adjoint(d, (1.0, 2.0, 3.0)).tolist() == [[0.0, 0.0, 0.0, 4.0, 2.0]]


@pytest.mark.parametrize("W", [9, 12, 37])
@pytest.mark.parametrize("taps", [O.SOBEL_D1, O.SOBEL_S5, "gauss"])
def test_correlate_adjoint_identity(W, taps):
    if taps == "gauss":
        taps = O.gaussian_taps(2.0)
    rng = np.random.default_rng(W)
    a = rng.normal(size=(3, W))
    b = rng.normal(size=(3, W))
    lhs = np.sum(O.correlate_x(a, taps) * b)
    rhs = np.sum(a * S.correlate_x_adjoint(b, taps))
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(a).sum() * np.abs(b).sum())


@pytest.mark.parametrize("shape", [(24, 31), (40, 17)])
def test_hessian_adjoint_identity(shape):
    rng = np.random.default_rng(sum(shape))
    a = rng.normal(size=shape)
    b = [rng.normal(size=shape) for _ in range(3)]
    Hs = O.hessian(a, 2.0)
    lhs = sum(np.sum(h * bb) for h, bb in zip(Hs, b))
    rhs = np.sum(a * S.hessian_adjoint(*b, 2.0))
    assert abs(lhs - rhs) <= 1e-12 * np.abs(a).sum() * max(np.abs(x).max() for x in b)


# ---------------------------------------------------------------- eigen adjoint

def test_eigen_vjp_matches_finite_differences():
    rng = np.random.default_rng(5)
    n = 400
    hxx, hyy = rng.normal(size=n), rng.normal(size=n)
    hxy = rng.choice([-1.0, 1.0], n) * rng.uniform(0.1, 1.0, n)    # away from the b = 0 wrap
    gk, gux, guy = rng.normal(size=(3, n))
    geo = S.geometry_from_hessian(hxx, hyy, hxy)
    dxx, dyy, dxy, dropped = S.eigen_vjp(geo, gk, gux, guy)
    assert dropped == 0

    def f(a, b, c):
        km, _, ux, uy = O.eigen(a, b, c)
        return gk * km + gux * ux + guy * uy

    h = 1e-6
    for got, pert in ((dxx, (1, 0, 0)), (dyy, (0, 1, 0)), (dxy, (0, 0, 1))):
        hp = [v + h * e for v, e in zip((hxx, hyy, hxy), pert)]
        hm = [v - h * e for v, e in zip((hxx, hyy, hxy), pert)]
        fd = (f(*hp) - f(*hm)) / (2 * h)
        np.testing.assert_allclose(got, fd, rtol=1e-6, atol=1e-8)


def test_eigen_vjp_drops_isotropic():
    geo = S.geometry_from_hessian(np.array([1.0, 1.0]), np.array([1.0, 1.0 + 1e-14]), np.array([0.0, 0.0]))
    _, _, _, dropped = S.eigen_vjp(geo, np.ones(2), np.ones(2), np.ones(2))
    assert dropped == 2


# ---------------------------------------------------------------- soft accumulator

def _brute_soft(xs, ys, w, ux, uy, W, H, r_lo, r_hi):
    """Definition written out: every cell receives w max(0, 1 - |dx|) max(0, 1 - |dy|)."""
    acc = np.zeros((r_hi - r_lo + 1, H, W))
    for p in range(len(xs)):
        for li, r in enumerate(range(r_lo, r_hi + 1)):
            for s in (1, -1):
                px, py = xs[p] + s * r * ux[p], ys[p] + s * r * uy[p]
                for cy in range(H):
                    for cx in range(W):
                        b = max(0.0, 1 - abs(px - cx)) * max(0.0, 1 - abs(py - cy))
                        acc[li, cy, cx] += w[p] * b
    return acc


def test_soft_accumulator_brute_force():
    rng = np.random.default_rng(11)
    W, H = 13, 11
    xs = np.array([2, 6, 10, 0, 12])
    ys = np.array([3, 5, 9, 0, 10])
    t = rng.uniform(-math.pi / 2, math.pi / 2, 5)
    ux, uy = -np.sin(t), np.cos(t)
    km = -rng.uniform(0.1, 2.0, 5)
    geo = dict(km=km, ux=ux, uy=uy)
    got = S.soft_accumulator(geo, xs, ys, W, H, 1, 6)
    ref = _brute_soft(xs, ys, -km, ux, uy, W, H, 1, 6)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


def test_soft_accumulator_axis_and_mass():
    W, H = 64, 64
    xs, ys = np.array([32]), np.array([30])
    geo = dict(km=np.array([-0.5]), ux=np.array([0.0]), uy=np.array([1.0]))
    acc = S.soft_accumulator(geo, xs, ys, W, H, 3, 9)
    for li, r in enumerate(range(3, 10)):
        expect = np.zeros((H, W))
        expect[30 + r, 32] += 0.5
        expect[30 - r, 32] += 0.5
        assert np.array_equal(acc[li], expect)
    # away from the border every splat keeps its whole weight: each level holds 2 sum w
    rng = np.random.default_rng(2)
    t = rng.uniform(-math.pi / 2, math.pi / 2, 30)
    xs, ys = rng.integers(20, 44, 30), rng.integers(20, 44, 30)
    geo = dict(km=-rng.uniform(0.1, 1, 30), ux=-np.sin(t), uy=np.cos(t))
    acc = S.soft_accumulator(geo, xs, ys, W, H, 5, 15)
    np.testing.assert_allclose(acc.sum(axis=(1, 2)), 2 * (-geo["km"]).sum(), rtol=1e-13)


def test_soft_vjp_matches_finite_differences():
    rng = np.random.default_rng(3)
    W, H, n = 40, 36, 25
    xs, ys = rng.integers(0, W, n), rng.integers(0, H, n)
    t = rng.uniform(-math.pi / 2, math.pi / 2, n)
    km = -rng.uniform(0.1, 1, n)
    G = rng.normal(size=(9, H, W))
    geo = dict(km=km, ux=-np.sin(t), uy=np.cos(t))
    gw, gux, guy = S.soft_accumulator_vjp(G, geo, xs, ys, W, H, 4, 12)

    def f(g):
        return float(np.sum(G * S.soft_accumulator(g, xs, ys, W, H, 4, 12)))

    h = 1e-6
    checked = skipped = 0
    for p in range(n):
        for key, got, sign in (("km", gw, -1.0), ("ux", gux, 1.0), ("uy", guy, 1.0)):
            vals = []
            for d in (h, -h, 0.0):
                g2 = {k: v.copy() for k, v in geo.items()}
                g2[key][p] += d
                vals.append(f(g2))
            fd = (vals[0] - vals[1]) / (2 * h)
            one_sided = ((vals[0] - vals[2]) / h, (vals[2] - vals[1]) / h)
            atol = 8 * EPS * max(abs(v) for v in vals) / h
            if abs(one_sided[0] - one_sided[1]) > 1e-3 * abs(fd) + 4 * atol:
                skipped += 1     # a bilinear kink within the step
                continue
            assert abs(sign * got[p] - fd) <= RTOL_FD * abs(fd) + atol, (p, key)
            checked += 1
    assert checked >= 70 and skipped <= 3


# ---------------------------------------------------------------- fit loss

def test_fit_loss_exact_on_noise_free_ring():
    theta = (40.3, 37.6, 20.45)
    img = S.render_ring(96, 96, theta, 1.5, 1.25, 0.2)
    L, A, B = S.fit_loss(img, theta, theta, 1.5)
    assert L <= 1e-24 and abs(A - 1.25) <= 1e-12 and abs(B - 0.2) <= 1e-12
    _, _, dI, dth = S.fit_loss_grad(img, theta, theta, 1.5)
    assert np.abs(dI).max() <= 1e-11 and np.abs(dth).max() <= 1e-9


def test_ring_window_symmetry_and_size():
    # an integer-centred window is symmetric under the dihedral group of the pixel grid
    xs, ys = S.ring_window((50.0, 50.0, 20.5), 1.5, 101, 101)
    m = np.zeros((101, 101), bool)
    m[ys, xs] = True
    assert np.array_equal(m, m.T) and np.array_equal(m, m[::-1]) and np.array_equal(m, m[:, ::-1])
    # pixel count ~ annulus area 2 pi r (2 (3 s + 2)), within the boundary's pixel count
    area = 2 * math.pi * 20.5 * 2 * 6.5
    assert abs(len(xs) - area) <= 2 * 2 * math.pi * (20.5 + 6.5)
    # clipped by the frame
    xs, ys = S.ring_window((2.0, 3.0, 10.0), 1.5, 30, 30)
    assert xs.min() == 0 and ys.min() == 0


def test_fit_loss_theta_gradient_50_rings():
    f = synth.config4(seed=3, n_frames=1, W=512, H=512, n_rings=80)[0]
    img = f.image.astype(np.float64)
    rng = np.random.default_rng(0)
    checked = 0
    for j in range(60):
        th0 = np.array([f.cx[j], f.cy[j], f.R[j]])
        th = th0 + rng.normal(0, 0.3, 3)
        _, _, _, g = S.fit_loss_grad(img, th, th0, 1.5)
        for k in range(3):
            e = np.zeros(3)
            e[k] = H_FD
            lp, lm = S.fit_loss(img, th + e, th0, 1.5)[0], S.fit_loss(img, th - e, th0, 1.5)[0]
            fd = (lp - lm) / (2 * H_FD)
            atol = 8 * EPS * max(lp, lm) / H_FD
            assert abs(g[k] - fd) <= RTOL_FD * abs(fd) + atol, (j, k, g[k], fd)
            checked += 1
    assert checked >= 150


# ---------------------------------------------------------------- the whole objective

@pytest.fixture(scope="module")
def small_case():
    """48x48 frame with two rings cut by the border, c1-like profile; radius bins 4..10."""
    W = H = 48
    truth = [(12.3, 20.6, 8.4), (40.2, 31.7, 9.3)]
    img = np.full((H, W), 0.2)
    for cx, cy, r in truth:
        img = img + S.render_ring(W, H, (cx, cy, r), 1.5, 1.0, 0.0)
    img = img + np.random.default_rng(9).normal(0, 0.05, img.shape)
    params = dict(O.DEFAULTS, r_min=5, r_max=9, k_threshold=-0.02)
    xs, ys, _, _, _ = O.ridges(img, params)
    r_lo, r_hi = S.levels(params)
    G = np.random.default_rng(10).normal(size=(r_hi - r_lo + 1, H, W))
    thetas0 = [np.array(t) for t in truth]
    thetas = [t + np.array([0.2, -0.3, 0.25]) for t in thetas0]
    return img, params, xs, ys, thetas, thetas0, G


def test_objective_image_gradient_finite_differences(small_case):
    img, params, xs, ys, thetas, thetas0, G = small_case
    assert len(xs) > 50
    dI, dth, dropped = S.objective_grad(img, params, xs, ys, thetas, thetas0, 1.5, G)
    assert dropped == 0
    H, W = img.shape
    yy, xx = np.mgrid[0:H, 0:W]
    border = np.minimum(np.minimum(xx, W - 1 - xx), np.minimum(yy, H - 1 - yy))
    pick = list(zip(*np.nonzero(border <= 3)))
    rng = np.random.default_rng(4)
    inner = list(zip(*np.nonzero(border > 3)))
    pick += [inner[i] for i in rng.choice(len(inner), 420, replace=False)]
    L0 = S.objective(img, params, xs, ys, thetas, thetas0, 1.5, G)
    checked = skipped = 0
    for y, x in pick:
        vals = []
        for d in (H_FD, -H_FD):
            im2 = img.copy()
            im2[y, x] += d
            vals.append(S.objective(im2, params, xs, ys, thetas, thetas0, 1.5, G))
        fd = (vals[0] - vals[1]) / (2 * H_FD)
        atol = 8 * EPS * max(abs(v) for v in vals + [L0]) / H_FD
        plus, minus = (vals[0] - L0) / H_FD, (L0 - vals[1]) / H_FD
        if abs(plus - minus) > 1e-3 * abs(fd) + 4 * atol:
            skipped += 1
            continue
        assert abs(dI[y, x] - fd) <= RTOL_FD * abs(fd) + atol, (y, x, dI[y, x], fd)
        checked += 1
    assert checked >= 1000 and skipped <= 0.02 * len(pick), (checked, skipped)


def test_objective_theta_gradient_finite_differences(small_case):
    img, params, xs, ys, thetas, thetas0, G = small_case
    _, dth, _ = S.objective_grad(img, params, xs, ys, thetas, thetas0, 1.5, G, lam=0.0)
    for j in range(len(thetas)):
        for k in range(3):
            e = np.zeros(3)
            e[k] = H_FD
            tp = [t + (e if i == j else 0) for i, t in enumerate(thetas)]
            tm = [t - (e if i == j else 0) for i, t in enumerate(thetas)]
            lp = S.objective(img, params, xs, ys, tp, thetas0, 1.5, G, lam=0.0)
            lm = S.objective(img, params, xs, ys, tm, thetas0, 1.5, G, lam=0.0)
            fd = (lp - lm) / (2 * H_FD)
            assert abs(dth[j, k] - fd) <= RTOL_FD * abs(fd) + 8 * EPS * max(lp, lm) / H_FD


# ---------------------------------------------------------------- refinement

def test_refine_converges_on_noise_free_ring():
    theta = np.array([40.3, 37.6, 20.45])
    img = S.render_ring(96, 96, theta, 1.5, 1.0, 0.2)
    for start in ((0.8, -0.6, 0.7), (-1.0, 0.5, -0.8), (0.3, 0.9, 1.2)):
        th, loss = S.refine(img, theta + np.array(start), 1.5, iters=20)
        assert np.abs(th - theta).max() <= 1e-6, (start, th - theta)
        assert loss <= 1e-12


def test_refine_lowers_loss_on_noisy_rings():
    f = synth.config4(seed=3, n_frames=1, W=256, H=256, n_rings=20)[0]
    img = f.image.astype(np.float64)
    rng = np.random.default_rng(1)
    err0 = err1 = 0.0
    for j in range(len(f.R)):
        truth = np.array([f.cx[j], f.cy[j], f.R[j]])
        th0 = truth + rng.normal(0, 0.5, 3)
        l0 = S.fit_loss(img, th0, th0, 1.5)[0]
        th, l1 = S.refine(img, th0, 1.5)
        assert l1 <= l0
        err0 += np.abs(th0 - truth).sum()
        err1 += np.abs(th - truth).sum()
    assert err1 < 0.2 * err0


def test_refine_rejects_a_step_that_raises_the_loss():
    # from this start the first damped Gauss-Newton step raises the loss (184.40 -> 185.24),
    # so it is not taken and the damping grows; later steps then make progress
    theta = np.array([40.3, 37.6, 20.45])
    img = S.render_ring(96, 96, theta, 1.5, 1.0, 0.2)
    start = theta + np.array([0.32201915, -1.17105765, -2.68243943])
    l0 = S.fit_loss(img, start, start, 1.5)[0]
    th1, l1 = S.refine(img, start, 1.5, iters=1)
    assert np.array_equal(th1, start) and l1 == l0
    th, l20 = S.refine(img, start, 1.5, iters=20)
    assert l20 < l0


def test_refine_infinite_tol_takes_exactly_one_step():
    # every update is within an infinite tolerance, so the first step (kept or not) is the last
    theta = np.array([40.3, 37.6, 20.45])
    img = S.render_ring(96, 96, theta, 1.5, 1.0, 0.2)
    for start in (theta + np.array([0.8, -0.6, 0.7]),                          # first step kept
                  theta + np.array([0.32201915, -1.17105765, -2.68243943])):   # first step refused
        th1, l1 = S.refine(img, start, 1.5, iters=1)
        th, l, n = S.refine(img, start, 1.5, iters=20, tol=np.inf, return_steps=True)
        assert n == 1 and np.array_equal(th, th1) and l == l1


def test_refine_tol_only_truncates_the_steps():
    # the stopping rule changes nothing but the step count: the same number of fixed steps
    # gives the same ring and loss, bit for bit; converged rings stop well before 20
    f = synth.config4(seed=3, n_frames=1, W=256, H=256, n_rings=12)[0]
    rng = np.random.default_rng(5)
    counts = []
    for j in range(len(f.R)):
        th0 = np.array([f.cx[j], f.cy[j], f.R[j]]) + rng.normal(0, 0.5, 3)
        th, l, n = S.refine(f.image, th0, 1.5, iters=20, tol=1e-8, return_steps=True)
        th_fixed, l_fixed = S.refine(f.image, th0, 1.5, iters=n)
        assert np.array_equal(th, th_fixed) and l == l_fixed
        th20, _ = S.refine(f.image, th0, 1.5, iters=20)
        assert np.abs(th - th20).max() <= 1e-7
        counts.append(n)
    assert max(counts) < 20 and np.mean(counts) < 10


def test_refine_tol_converges_on_noise_free_ring():
    theta = np.array([40.3, 37.6, 20.45])
    img = S.render_ring(96, 96, theta, 1.5, 1.0, 0.2)
    for start in ((0.8, -0.6, 0.7), (-1.0, 0.5, -0.8), (0.3, 0.9, 1.2)):
        th, loss, n = S.refine(img, theta + np.array(start), 1.5, iters=20, tol=1e-8, return_steps=True)
        assert n < 10 and np.abs(th - theta).max() <= 1e-6 and loss <= 1e-12


def test_refine_singular_steps_do_not_stop():
    # a zero image: A = 0, so J = 0 and every system is singular; no step has an update,
    # none ends the loop, the ring stays where it started
    img = np.zeros((64, 64))
    start = np.array([30.2, 31.7, 12.4])
    th, loss, n = S.refine(img, start, 1.5, iters=7, tol=np.inf, return_steps=True)
    assert n == 7 and np.array_equal(th, start) and loss == 0.0
