"""FP64 oracle of the differentiable extension: soft accumulator, ring-profile fit loss, their
adjoints and the gradient refinement of rings.

TEST INFRASTRUCTURE ONLY, like ridge_hough.py: only the tests, the smoke check and the
benchmark's CPU-baseline leg may use it, and it shares no code with the HIP path.

The paper has no differentiable path; what follows fixes one, built on the plain method's
quantities (readings):

  soft accumulator  A~_r(c) = sum_{p in R} sum_{s = +-1} w_p beta(p + s r u_p - c) with the
                    bilinear splat beta(d) = max(0, 1 - |dx|) max(0, 1 - |dy|), the weight
                    w_p = -k_-(p) and u_p the continuous X_-(p) (not the fixed-point code).
                    R is the plain method's ridge set, held fixed (the selection is not
                    differentiable); levels r_min - 1 .. r_max + 1 as the votes; cells off the
                    frame are dropped.
  fit loss          L_j = sum_{p in W_j} (I(p) - B_j - A_j g_j(p))^2 with the ring profile
                    g_j(p) = exp(-(|p - c_j| - r_j)^2 / (2 s^2)) and (A_j, B_j) the linear least
                    squares at the current (c_j, r_j).  The window
                    W_j = {p : | |p - c0_j| - r0_j | <= 3 s + 2} is fixed by the starting ring.
  check objective   L = sum_j L_j + lam <G, A~>.
  refinement        damped Gauss-Newton (Levenberg-Marquardt) on (cx, cy, r) per ring with
                    (A, B) eliminated (solved in closed form at every point).

The Hessian is the plain method's (Methods, "Algorithm implementation": Gaussian smoothing,
then 5x5 second-order Sobel kernels / 64, every 1D correlation with its own reflect-101
border), so its adjoint is the chain of the transposed 1D correlations, each followed by
folding the border halo back onto the mirrored pixels.
"""
from __future__ import annotations

import math

import numpy as np

from . import ridge_hough as O

ISO_REL = 1e-12   # eigenvector term dropped where d = |k_+ - k_-| / 2 <= ISO_REL max|H|


# --------------------------------------------------------------------------------------
# Adjoint of the Hessian operator I -> (Ixx, Iyy, Ixy)
# --------------------------------------------------------------------------------------

def correlate_x_adjoint(d: np.ndarray, taps) -> np.ndarray:
    """Transpose of ridge_hough.correlate_x:
    out(y, q) = sum over (x, j) with reflect101(x + j - R) = q of taps[j] d(y, x).
    The extended-domain sums are formed first, then each extended column is added onto the
    frame column it mirrors to."""
    taps = np.asarray(taps, dtype=np.float64)
    R = len(taps) // 2
    H, W = d.shape
    ext = np.zeros((H, W + 2 * R))
    for j, t in enumerate(taps):
        ext[:, j:j + W] += t * d           # x + j - R is extended column x + j
    cols = O.reflect101(np.arange(-R, W + R), W)
    out = np.zeros((H, W))
    for e in range(W + 2 * R):
        out[:, cols[e]] += ext[:, e]
    return out


def correlate_y_adjoint(d: np.ndarray, taps) -> np.ndarray:
    return correlate_x_adjoint(d.T, taps).T


def hessian_adjoint(dxx, dyy, dxy, sigma):
    """dI = transpose of ridge_hough.hessian applied to (dIxx, dIyy, dIxy)."""
    dG = (correlate_x_adjoint(correlate_y_adjoint(dxx, O.SOBEL_S5), O.SOBEL_D2)
          + correlate_x_adjoint(correlate_y_adjoint(dyy, O.SOBEL_D2), O.SOBEL_S5)
          + correlate_x_adjoint(correlate_y_adjoint(dxy, O.SOBEL_D1), O.SOBEL_D1)) / 64.0
    g = O.gaussian_taps(sigma)
    return correlate_x_adjoint(correlate_y_adjoint(dG, g), g)


# --------------------------------------------------------------------------------------
# Soft accumulator
# --------------------------------------------------------------------------------------

def ridge_geometry(img, params, xs, ys):
    """Hessian entries, k_-, k_+ and the continuous X_- = (ux, uy) at the given pixels."""
    p = dict(O.DEFAULTS, **params)
    Ixx, Iyy, Ixy = O.hessian(np.asarray(img, dtype=np.float64), O.f32(p["sigma_smooth"]))
    return geometry_from_hessian(Ixx[ys, xs], Iyy[ys, xs], Ixy[ys, xs])


def geometry_from_hessian(hxx, hyy, hxy):
    km, kp, ux, uy = O.eigen(hxx, hyy, hxy)
    return dict(hxx=hxx, hyy=hyy, hxy=hxy, km=km, kp=kp, ux=ux, uy=uy)


def levels(params):
    p = dict(O.DEFAULTS, **params)
    return int(p["r_min"]) - 1, int(p["r_max"]) + 1


def _splat(xs, ys, ux, uy, r, s):
    """Splat position p + s r u (x then y) and its bilinear cell corner and fractions."""
    px = xs + s * r * ux
    py = ys + s * r * uy
    i0 = np.floor(px)
    j0 = np.floor(py)
    return i0.astype(np.int64), j0.astype(np.int64), px - i0, py - j0


CORNERS = ((0, 0), (1, 0), (0, 1), (1, 1))


def soft_accumulator(geo, xs, ys, W, H, r_lo, r_hi):
    """A~ as float64 of shape (L, H, W), L = r_hi - r_lo + 1."""
    L = r_hi - r_lo + 1
    acc = np.zeros((L, H, W))
    w = -geo["km"]
    for li in range(L):
        r = r_lo + li
        for s in (1.0, -1.0):
            i0, j0, fx, fy = _splat(xs, ys, geo["ux"], geo["uy"], r, s)
            for di, dj in CORNERS:
                beta = (fx if di else 1.0 - fx) * (fy if dj else 1.0 - fy)
                ci, cj = i0 + di, j0 + dj
                ok = (ci >= 0) & (ci < W) & (cj >= 0) & (cj < H)
                np.add.at(acc[li], (cj[ok], ci[ok]), (w * beta)[ok])
    return acc


def soft_accumulator_vjp(G, geo, xs, ys, W, H, r_lo, r_hi):
    """Gradients of <G, A~> with respect to w_p and u_p: (gw, gux, guy).  Inside a cell the
    splat is bilinear, so d beta / d px = +-(1 - fy or fy) and the chain through
    px = x + s r ux gives the factor s r."""
    w = -geo["km"]
    n = len(xs)
    gw, gux, guy = np.zeros(n), np.zeros(n), np.zeros(n)
    for li in range(r_hi - r_lo + 1):
        r = r_lo + li
        for s in (1.0, -1.0):
            i0, j0, fx, fy = _splat(xs, ys, geo["ux"], geo["uy"], r, s)
            for di, dj in CORNERS:
                bx = fx if di else 1.0 - fx
                by = fy if dj else 1.0 - fy
                ci, cj = i0 + di, j0 + dj
                ok = (ci >= 0) & (ci < W) & (cj >= 0) & (cj < H)
                gv = np.zeros(n)
                gv[ok] = G[li, cj[ok], ci[ok]]
                gw += gv * bx * by
                gux += w * gv * (1.0 if di else -1.0) * by * s * r
                guy += w * gv * bx * (1.0 if dj else -1.0) * s * r
    return gw, gux, guy


def eigen_vjp(geo, gk, gux, guy):
    """Adjoint of (Ixx, Iyy, Ixy) -> (k_-, X_-) given dL/dk_- and dL/dX_-.
    First-order perturbation of a symmetric 2x2 matrix: dk_- = X_-^T dH X_- and
    dX_- = (X_+^T dH X_- / (k_- - k_+)) X_+ with X_+ = (uy, -ux); Ixy stands for both
    off-diagonal entries.  Where d <= ISO_REL max|H| (near-isotropic) the X_- term is
    dropped; returns (dxx, dyy, dxy, number dropped)."""
    ux, uy = geo["ux"], geo["uy"]
    vx, vy = uy, -ux
    dxx = gk * ux * ux
    dyy = gk * uy * uy
    dxy = gk * 2.0 * ux * uy
    gap = geo["km"] - geo["kp"]
    scale = np.maximum(np.maximum(np.abs(geo["hxx"]), np.abs(geo["hyy"])), np.abs(geo["hxy"]))
    ok = 0.5 * np.abs(gap) > ISO_REL * scale
    alpha = np.where(ok, (gux * vx + guy * vy) / np.where(ok, gap, 1.0), 0.0)
    dxx = dxx + alpha * vx * ux
    dyy = dyy + alpha * vy * uy
    dxy = dxy + alpha * (vx * uy + vy * ux)
    return dxx, dyy, dxy, int(np.count_nonzero(~ok))


# --------------------------------------------------------------------------------------
# Ring-profile fit loss
# --------------------------------------------------------------------------------------

def window_halfwidth(s):
    return 3.0 * s + 2.0


def ring_window(theta0, s, W, H):
    """Pixels of W_j, ascending (y, x).  Membership is decided in float64 as
    |sqrt(dx*dx + dy*dy) - r0| <= 3 s + 2 with dx = x - cx0, dy = y - cy0, every operation
    rounded separately."""
    cx, cy, r = (float(v) for v in theta0)
    m = window_halfwidth(s)
    ext = r + m
    x0, x1 = max(0, int(math.floor(cx - ext))), min(W - 1, int(math.ceil(cx + ext)))
    y0, y1 = max(0, int(math.floor(cy - ext))), min(H - 1, int(math.ceil(cy + ext)))
    if x1 < x0 or y1 < y0:
        e = np.zeros(0, dtype=np.int64)
        return e, e
    yy, xx = np.mgrid[y0:y1 + 1, x0:x1 + 1]
    dx = xx - cx
    dy = yy - cy
    rho = np.sqrt(dx * dx + dy * dy)
    keep = np.abs(rho - r) <= m
    return xx[keep].astype(np.int64), yy[keep].astype(np.int64)


def profile(xs, ys, theta, s):
    cx, cy, r = (float(v) for v in theta)
    dx = xs - cx
    dy = ys - cy
    rho = np.sqrt(dx * dx + dy * dy)
    g = np.exp(-((rho - r) ** 2) / (2.0 * s * s))
    return g, rho


def profile_jacobian(xs, ys, theta, s, g, rho):
    """dg/d(cx, cy, r), shape (n, 3); at rho = 0 the centre derivatives are taken as 0."""
    cx, cy, r = (float(v) for v in theta)
    dg_drho = -g * (rho - r) / (s * s)
    safe = np.where(rho > 0, rho, 1.0)
    return np.stack([dg_drho * (-(xs - cx) / safe), dg_drho * (-(ys - cy) / safe), -dg_drho], 1)


def fit_ab(I_win, g):
    """Least squares of I ~ B + A g by Cramer's rule on the 2x2 normal equations.  READING:
    an empty window gives (0, 0); a singular system (all g equal) gives A = 0, B = mean I."""
    n = float(len(g))
    if n == 0:
        return 0.0, 0.0
    Sg, Sgg = float(g.sum()), float(np.dot(g, g))
    SI, SIg = float(I_win.sum()), float(np.dot(I_win, g))
    det = Sgg * n - Sg * Sg
    if det == 0.0:
        return 0.0, SI / n
    return (SIg * n - Sg * SI) / det, (Sgg * SI - Sg * SIg) / det


def _window(img, theta0, s):
    H, W = img.shape
    xs, ys = ring_window(theta0, s, W, H)
    return xs, ys, np.asarray(img, dtype=np.float64)[ys, xs]


def fit_loss(img, theta, theta0, s):
    """(L_j, A_j, B_j) of one ring."""
    xs, ys, I_win = _window(img, theta0, s)
    g, _ = profile(xs, ys, theta, s)
    A, B = fit_ab(I_win, g)
    e = I_win - B - A * g
    return float(np.dot(e, e)), A, B


def fit_loss_grad(img, theta, theta0, s):
    """Window pixels (xs, ys), dL_j/dI on them and dL_j/dtheta.  (A, B) sit at their
    least-squares optimum, so their own variation contributes nothing (envelope theorem)."""
    xs, ys, I_win = _window(img, theta0, s)
    g, rho = profile(xs, ys, theta, s)
    A, B = fit_ab(I_win, g)
    e = I_win - B - A * g
    J = profile_jacobian(xs, ys, theta, s, g, rho)
    return xs, ys, 2.0 * e, (-2.0 * A * e) @ J


# --------------------------------------------------------------------------------------
# The check objective and its gradient
# --------------------------------------------------------------------------------------

def objective(img, params, xs, ys, thetas, thetas0, s, G, lam=1.0):
    img = np.asarray(img, dtype=np.float64)
    H, W = img.shape
    total = sum(fit_loss(img, th, th0, s)[0] for th, th0 in zip(thetas, thetas0))
    if lam != 0.0 and len(xs):
        r_lo, r_hi = levels(params)
        geo = ridge_geometry(img, params, xs, ys)
        total += lam * float(np.sum(G * soft_accumulator(geo, xs, ys, W, H, r_lo, r_hi)))
    return total


def soft_image_grad(img, params, xs, ys, G):
    """d<G, A~>/dI and the number of near-isotropic ridge pixels whose X_- term was dropped."""
    img = np.asarray(img, dtype=np.float64)
    H, W = img.shape
    p = dict(O.DEFAULTS, **params)
    r_lo, r_hi = levels(p)
    geo = ridge_geometry(img, p, xs, ys)
    gw, gux, guy = soft_accumulator_vjp(G, geo, xs, ys, W, H, r_lo, r_hi)
    dxx, dyy, dxy, dropped = eigen_vjp(geo, -gw, gux, guy)     # w = -k_-
    planes = [np.zeros((H, W)) for _ in range(3)]
    for pl, v in zip(planes, (dxx, dyy, dxy)):
        pl[ys, xs] = v
    return hessian_adjoint(*planes, O.f32(p["sigma_smooth"])), dropped


def objective_grad(img, params, xs, ys, thetas, thetas0, s, G, lam=1.0):
    """(dL/dI, dL/dtheta of shape (m, 3), dropped isotropic count)."""
    img = np.asarray(img, dtype=np.float64)
    dI = np.zeros(img.shape)
    dth = np.zeros((len(thetas), 3))
    for j, (th, th0) in enumerate(zip(thetas, thetas0)):
        wx, wy, dv, dt = fit_loss_grad(img, th, th0, s)
        np.add.at(dI, (wy, wx), dv)
        dth[j] = dt
    dropped = 0
    if lam != 0.0 and len(xs):
        dS, dropped = soft_image_grad(img, params, xs, ys, G)
        dI += lam * dS
    return dI, dth, dropped


# --------------------------------------------------------------------------------------
# Gradient refinement of a ring: Levenberg-Marquardt on (cx, cy, r)
# --------------------------------------------------------------------------------------

LM_LAMBDA0 = 1e-3
LM_DOWN = 1.0 / 3.0
LM_UP = 4.0


def refine(img, theta0, s, iters=20, tol=0.0, return_steps=False):
    """(theta, loss) after at most `iters` Levenberg-Marquardt steps from theta0.  Each step
    takes the residual e = I - B - A g and its Jacobian J = -A dg/dtheta at the current ring
    with (A, B) at their optimum there, solves (J^T J + lam diag(J^T J)) d = -J^T e, and keeps
    theta + d only if the loss with (A, B) re-solved is lower; lam is divided by 3 after a
    kept step and multiplied by 4 otherwise (also when the system is singular).

    READING (convergence, an addition to the fixed step count): the loop ends after a step
    whose solved update has every component at most `tol` in magnitude, kept or not; a step
    whose system is singular has no update and does not end it.  tol = 0 stops only on an
    exactly zero update, after which every further step would repeat it unchanged.  With
    return_steps the number of steps taken comes third."""
    xs, ys, I_win = _window(img, theta0, s)

    def evaluate(th):
        g, rho = profile(xs, ys, th, s)
        A, B = fit_ab(I_win, g)
        e = I_win - B - A * g
        return float(np.dot(e, e)), g, rho, A, e

    th = np.array(theta0, dtype=np.float64)
    lam = LM_LAMBDA0
    loss, g, rho, A, e = evaluate(th)
    steps = 0
    for _ in range(iters):
        steps += 1
        J = -A * profile_jacobian(xs, ys, th, s, g, rho)
        M = J.T @ J
        try:
            d = np.linalg.solve(M + lam * np.diag(np.diag(M)), -(J.T @ e))
        except np.linalg.LinAlgError:
            lam *= LM_UP
            continue
        cand = th + d
        l2, g2, rho2, A2, e2 = evaluate(cand)
        if l2 < loss:
            th, loss, g, rho, A, e = cand, l2, g2, rho2, A2, e2
            lam *= LM_DOWN
        else:
            lam *= LM_UP
        if np.max(np.abs(d)) <= tol:
            break
    return (th, loss, steps) if return_steps else (th, loss)


def render_ring(W, H, theta, s, A, B):
    """Noise-free ring with exactly the fit-loss profile (a test fixture)."""
    yy, xx = np.mgrid[0:H, 0:W]
    g, _ = profile(xx.astype(np.float64), yy.astype(np.float64), theta, s)
    return B + A * g
