// Ring-profile fit of the differentiable extension: per ring j the loss
//   L_j = sum_{p in W_j} (I(p) - B_j - A_j g_j(p))^2,  g_j(p) = exp(-(|p - c_j| - r_j)^2 / (2 s^2)),
// with (A_j, B_j) the linear least-squares fit at the current ring and the window
// W_j = {p : | |p - c0_j| - r0_j | <= 3 s + 2} fixed by the starting ring; its gradient with
// respect to the image and to (cx, cy, r); and Levenberg-Marquardt refinement of (cx, cy, r)
// with (A, B) eliminated.  The paper fits circles to each classified ridge set (Results,
// "Directed ridge detection & votes collection"); this profile fit refines those circles on
// the image itself.
//
// One workgroup per ring.  Every pass walks the window's bounding box; membership is decided
// in fp64 with separately rounded operations, so each pixel is in or out exactly as a float64
// reference decides.  All sums are fp64.
#include "rd_internal.h"

namespace rd {
namespace {

constexpr int NT = 256;
constexpr int NW = NT / 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sums K values over the workgroup; every thread gets the totals.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* sred) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double t = wave_sum(v[k]);
        if (lane == 0) sred[wave * K + k] = t;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) t += sred[w * K + k];
        v[k] = t;
    }
    __syncthreads();
}

// fmin / fmax return the other operand for a NaN, so the result is always in [lo, hi].
__device__ __forceinline__ double clampd(double v, double lo, double hi) { return fmin(fmax(v, lo), hi); }

struct Window {
    int x0, y0, bw, bh;
    double cx0, cy0, r0, m;
};

__device__ __forceinline__ Window make_window(const double* th0, double m, int W, int H) {
    Window w;
    w.cx0 = th0[0];
    w.cy0 = th0[1];
    w.r0 = th0[2];
    w.m = m;
    // bounding box clamped to the frame in floating point first, so that any input (huge or
    // not finite) converts to an in-frame integer range; membership then decides
    const double ext = __dadd_rn(w.r0, m);
    const int x0 = static_cast<int>(clampd(floor(__dsub_rn(w.cx0, ext)), 0.0, W - 1.0));
    const int x1 = static_cast<int>(clampd(ceil(__dadd_rn(w.cx0, ext)), 0.0, W - 1.0));
    const int y0 = static_cast<int>(clampd(floor(__dsub_rn(w.cy0, ext)), 0.0, H - 1.0));
    const int y1 = static_cast<int>(clampd(ceil(__dadd_rn(w.cy0, ext)), 0.0, H - 1.0));
    w.x0 = x0;
    w.y0 = y0;
    w.bw = x1 >= x0 ? x1 - x0 + 1 : 0;
    w.bh = y1 >= y0 ? y1 - y0 + 1 : 0;
    return w;
}

__device__ __forceinline__ bool in_window(const Window& w, int x, int y) {
    const double dx = __dsub_rn(static_cast<double>(x), w.cx0);
    const double dy = __dsub_rn(static_cast<double>(y), w.cy0);
    const double rho = __dsqrt_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)));
    return fabs(__dsub_rn(rho, w.r0)) <= w.m;
}

__device__ __forceinline__ double pixel(const RingFrame& f, int x, int y) {
    const char* row = static_cast<const char*>(f.img) + static_cast<int64_t>(y) * f.pitch;
    return f.dtype == RD_U16 ? static_cast<double>(reinterpret_cast<const uint16_t*>(row)[x])
                             : static_cast<double>(reinterpret_cast<const float*>(row)[x]);
}

struct Prof {
    double g, rho, dgdrho;
};

__device__ __forceinline__ Prof profile(double cx, double cy, double r, double inv2s2, double invs2, int x, int y) {
    Prof p;
    const double dx = x - cx, dy = y - cy;
    p.rho = sqrt(dx * dx + dy * dy);
    const double t = p.rho - r;
    p.g = exp(-(t * t) * inv2s2);
    p.dgdrho = -p.g * t * invs2;
    return p;
}

// Closed-form (A, B) from the sums n, Sg, Sgg, SI, SIg (Cramer's rule on the 2x2 normal
// equations); an empty window gives (0, 0), a singular system A = 0, B = mean I.
__device__ __forceinline__ void solve_ab(const double* s, double& A, double& B) {
    const double n = s[0], Sg = s[1], Sgg = s[2], SI = s[3], SIg = s[4];
    if (n == 0.0) {
        A = 0.0;
        B = 0.0;
        return;
    }
    const double det = Sgg * n - Sg * Sg;
    if (det == 0.0) {
        A = 0.0;
        B = SI / n;
        return;
    }
    A = (SIg * n - Sg * SI) / det;
    B = (Sgg * SI - Sg * SIg) / det;
}

// (A, B) at ring th; returns nothing, fills A, B.
__device__ void fit_ab(const RingFrame& f, const Window& w, const double* th, double inv2s2, double invs2,
                       double* sred, double& A, double& B) {
    double s[5] = {0, 0, 0, 0, 0};
    const int64_t nbox = static_cast<int64_t>(w.bw) * w.bh;
    for (int64_t i = threadIdx.x; i < nbox; i += NT) {
        const int y = w.y0 + static_cast<int>(i / w.bw), x = w.x0 + static_cast<int>(i % w.bw);
        if (!in_window(w, x, y)) continue;
        const double I = pixel(f, x, y);
        const Prof p = profile(th[0], th[1], th[2], inv2s2, invs2, x, y);
        s[0] += 1.0;
        s[1] += p.g;
        s[2] += p.g * p.g;
        s[3] += I;
        s[4] += I * p.g;
    }
    block_sum<5>(s, sred);
    solve_ab(s, A, B);
}

__device__ double residual_loss(const RingFrame& f, const Window& w, const double* th, double A, double B,
                                double inv2s2, double invs2, double* sred) {
    double s[1] = {0.0};
    const int64_t nbox = static_cast<int64_t>(w.bw) * w.bh;
    for (int64_t i = threadIdx.x; i < nbox; i += NT) {
        const int y = w.y0 + static_cast<int>(i / w.bw), x = w.x0 + static_cast<int>(i % w.bw);
        if (!in_window(w, x, y)) continue;
        const Prof p = profile(th[0], th[1], th[2], inv2s2, invs2, x, y);
        const double e = pixel(f, x, y) - B - A * p.g;
        s[0] += e * e;
    }
    block_sum<1>(s, sred);
    return s[0];
}

__global__ __launch_bounds__(NT) void k_fit_loss(RingArgs a, int backward) {
    __shared__ double sred[NW * 8];
    const double inv2s2 = 1.0 / (2.0 * a.s * a.s), invs2 = 1.0 / (a.s * a.s);
    for (int64_t j = blockIdx.x; j < a.m; j += gridDim.x) {
        const int fi = a.frame_of ? a.frame_of[j] : 0;
        if (fi < 0 || fi >= a.nframes) {
            if (threadIdx.x == 0) {
                if (backward) {
                    for (int c = 0; c < 3; ++c) a.grad_theta[3 * j + c] = __builtin_nan("");
                } else {
                    a.loss[j] = __builtin_nan("");
                    if (a.ab) a.ab[2 * j] = a.ab[2 * j + 1] = __builtin_nan("");
                }
            }
            continue;
        }
        const RingFrame f = a.frames[fi];
        const Window w = make_window(a.theta0 + 3 * j, a.halfwidth, f.W, f.H);
        const double th[3] = {a.theta[3 * j], a.theta[3 * j + 1], a.theta[3 * j + 2]};
        double A, B;
        fit_ab(f, w, th, inv2s2, invs2, sred, A, B);
        if (!backward) {
            const double L = residual_loss(f, w, th, A, B, inv2s2, invs2, sred);
            if (threadIdx.x == 0) {
                a.loss[j] = L;
                if (a.ab) {
                    a.ab[2 * j] = A;
                    a.ab[2 * j + 1] = B;
                }
            }
            continue;
        }
        // dL/dI = 2 e on the window; dL/dtheta = sum -2 A e dg/dtheta ((A, B) at their optimum)
        const double gl = a.grad_loss[j];
        double s[3] = {0, 0, 0};
        const int64_t nbox = static_cast<int64_t>(w.bw) * w.bh;
        for (int64_t i = threadIdx.x; i < nbox; i += NT) {
            const int y = w.y0 + static_cast<int>(i / w.bw), x = w.x0 + static_cast<int>(i % w.bw);
            if (!in_window(w, x, y)) continue;
            const Prof p = profile(th[0], th[1], th[2], inv2s2, invs2, x, y);
            const double e = pixel(f, x, y) - B - A * p.g;
            if (a.grad_img) atomicAdd(&a.grad_img[static_cast<int64_t>(y) * f.W + x], static_cast<float>(gl * 2.0 * e));
            const double safe = p.rho > 0.0 ? p.rho : 1.0;
            const double c = -2.0 * A * e * p.dgdrho;
            s[0] += c * (-(x - th[0]) / safe);
            s[1] += c * (-(y - th[1]) / safe);
            s[2] -= c;
        }
        block_sum<3>(s, sred);
        if (threadIdx.x == 0) {
            a.grad_theta[3 * j] = gl * s[0];
            a.grad_theta[3 * j + 1] = gl * s[1];
            a.grad_theta[3 * j + 2] = gl * s[2];
        }
    }
}

// Solves the 3x3 system M d = b by Gaussian elimination with partial pivoting; false when a
// pivot is exactly zero.
__device__ bool solve3(double M[3][3], double b[3], double d[3]) {
    for (int k = 0; k < 3; ++k) {
        int p = k;
        for (int i = k + 1; i < 3; ++i)
            if (fabs(M[i][k]) > fabs(M[p][k])) p = i;
        if (M[p][k] == 0.0) return false;
        if (p != k) {
            for (int c = 0; c < 3; ++c) {
                const double t = M[k][c];
                M[k][c] = M[p][c];
                M[p][c] = t;
            }
            const double t = b[k];
            b[k] = b[p];
            b[p] = t;
        }
        for (int i = k + 1; i < 3; ++i) {
            const double l = M[i][k] / M[k][k];
            for (int c = k; c < 3; ++c) M[i][c] -= l * M[k][c];
            b[i] -= l * b[k];
        }
    }
    for (int k = 2; k >= 0; --k) {
        double t = b[k];
        for (int c = k + 1; c < 3; ++c) t -= M[k][c] * d[c];
        d[k] = t / M[k][k];
    }
    return true;
}

__global__ __launch_bounds__(NT) void k_refine(RingArgs a) {
    __shared__ double sred[NW * 9];
    const double inv2s2 = 1.0 / (2.0 * a.s * a.s), invs2 = 1.0 / (a.s * a.s);
    for (int64_t j = blockIdx.x; j < a.m; j += gridDim.x) {
        const int fi = a.frame_of ? a.frame_of[j] : 0;
        if (fi < 0 || fi >= a.nframes) {
            if (threadIdx.x == 0) {
                for (int c = 0; c < 3; ++c) a.theta_out[3 * j + c] = __builtin_nan("");
                if (a.loss) a.loss[j] = __builtin_nan("");
            }
            continue;
        }
        const RingFrame f = a.frames[fi];
        const Window w = make_window(a.theta0 + 3 * j, a.halfwidth, f.W, f.H);
        double th[3] = {a.theta0[3 * j], a.theta0[3 * j + 1], a.theta0[3 * j + 2]};
        double lam = a.lam0;
        double A, B;
        fit_ab(f, w, th, inv2s2, invs2, sred, A, B);
        double loss = residual_loss(f, w, th, A, B, inv2s2, invs2, sred);
        const int64_t nbox = static_cast<int64_t>(w.bw) * w.bh;
        for (int it = 0; it < a.iters; ++it) {
            // J = -A dg/dtheta and e at the current ring: sums of J^T J (6) and J^T e (3)
            double s[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            for (int64_t i = threadIdx.x; i < nbox; i += NT) {
                const int y = w.y0 + static_cast<int>(i / w.bw), x = w.x0 + static_cast<int>(i % w.bw);
                if (!in_window(w, x, y)) continue;
                const Prof p = profile(th[0], th[1], th[2], inv2s2, invs2, x, y);
                const double e = pixel(f, x, y) - B - A * p.g;
                const double safe = p.rho > 0.0 ? p.rho : 1.0;
                const double j0 = -A * p.dgdrho * (-(x - th[0]) / safe);
                const double j1 = -A * p.dgdrho * (-(y - th[1]) / safe);
                const double j2 = -A * -p.dgdrho;
                s[0] += j0 * j0;
                s[1] += j0 * j1;
                s[2] += j0 * j2;
                s[3] += j1 * j1;
                s[4] += j1 * j2;
                s[5] += j2 * j2;
                s[6] += j0 * e;
                s[7] += j1 * e;
                s[8] += j2 * e;
            }
            block_sum<9>(s, sred);
            // (J^T J + lam diag(J^T J)) d = -J^T e, solved redundantly by every thread
            double M[3][3] = {{s[0] + lam * s[0], s[1], s[2]},
                              {s[1], s[3] + lam * s[3], s[4]},
                              {s[2], s[4], s[5] + lam * s[5]}};
            double b[3] = {-s[6], -s[7], -s[8]};
            double d[3] = {0, 0, 0};
            if (!solve3(M, b, d)) {
                lam *= a.lam_up;
                continue;
            }
            const double cand[3] = {th[0] + d[0], th[1] + d[1], th[2] + d[2]};
            double A2, B2;
            fit_ab(f, w, cand, inv2s2, invs2, sred, A2, B2);
            const double l2 = residual_loss(f, w, cand, A2, B2, inv2s2, invs2, sred);
            if (l2 < loss) {
                th[0] = cand[0];
                th[1] = cand[1];
                th[2] = cand[2];
                loss = l2;
                A = A2;
                B = B2;
                lam *= a.lam_down;
            } else {
                lam *= a.lam_up;
            }
        }
        if (threadIdx.x == 0) {
            a.theta_out[3 * j] = th[0];
            a.theta_out[3 * j + 1] = th[1];
            a.theta_out[3 * j + 2] = th[2];
            if (a.loss) a.loss[j] = loss;
        }
    }
}

int ring_grid(int64_t m) { return static_cast<int>(m < 65536 ? m : 65536); }

}  // namespace

hipError_t launch_fit_loss(const RingArgs& a, bool backward, hipStream_t s) {
    if (a.m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fit_loss, dim3(ring_grid(a.m)), dim3(NT), 0, s, a, backward ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_refine(const RingArgs& a, hipStream_t s) {
    if (a.m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_refine, dim3(ring_grid(a.m)), dim3(NT), 0, s, a);
    return hipGetLastError();
}

}  // namespace rd
