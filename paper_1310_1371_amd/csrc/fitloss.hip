// Ring-profile fit of the differentiable extension: per ring j the loss
//   L_j = sum_{p in W_j} (I(p) - B_j - A_j g_j(p))^2,  g_j(p) = exp(-(|p - c_j| - r_j)^2 / (2 s^2)),
// with (A_j, B_j) the linear least-squares fit at the current ring and the window
// W_j = {p : | |p - c0_j| - r0_j | <= 3 s + 2} fixed by the starting ring; its gradient with
// respect to the image and to (cx, cy, r); and Levenberg-Marquardt refinement of (cx, cy, r)
// with (A, B) eliminated.  The paper fits circles to each classified ridge set (Results,
// "Directed ridge detection & votes collection"); this profile fit refines those circles on
// the image itself.
//
// One workgroup per ring.  The window's members are found once, by walking its bounding box
// with membership decided in fp64 with separately rounded operations (each pixel is in or out
// exactly as a float64 reference decides), and compacted into LDS with their intensities;
// every later pass reads the LDS list.  Windows larger than the list fall back to walking the
// box on every pass.  All sums are fp64.
//
// Refinement pass: one sweep per LM step.  With d = dg/dtheta, the sweep accumulates
//   sum g, sum g^2, sum I g, sum d d^T, sum d I, sum d, sum d g
// (n, sum I, sum I^2 once per ring).  From these, in closed form: (A, B); the loss at the
// optimum L = sum I^2 - A sum I g - B sum I (the residual is orthogonal to 1 and g);
// J^T J = A^2 sum d d^T and -J^T e = A (sum d I - B sum d - A sum d g) for J = -A d.
#include "rd_internal.h"

namespace rd {
namespace {

constexpr int NT = 256;
constexpr int NW = NT / 64;
// window members held in LDS (8 bytes each): the loss kernel's list keeps 3 workgroups per CU;
// the refinement kernel (2 per CU by its registers) lists rings up to r ~ 90 at s = 1.5; above
// 64 KiB per workgroup the compiler would plan for one workgroup per CU and take more registers
constexpr int WCAP_LOSS = 6144;
constexpr int WCAP_REFINE = 7936;

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

__device__ __forceinline__ float pixel(const RingFrame& f, int x, int y) {
    const char* row = static_cast<const char*>(f.img) + static_cast<int64_t>(y) * f.pitch;
    return f.dtype == RD_U16 ? static_cast<float>(reinterpret_cast<const uint16_t*>(row)[x])
                             : reinterpret_cast<const float*>(row)[x];
}

// The window's members: either compacted in LDS (listed) or found again on every pass.
struct Members {
    const uint32_t* pos;   // (x - x0) | (y - y0) << 16
    const float* val;
    int n;
    bool listed;
};

// c (optional) receives this thread's part of n, sum I, sum I^2 over the members it lists;
// when the window does not fit the list, the caller sums them by a walk of the box.
template <int WCAP>
__device__ Members build_members(const RingFrame& f, const Window& w, uint32_t* sPos, float* sVal,
                                 uint32_t* sCnt, double* c = nullptr) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t nbox = static_cast<int64_t>(w.bw) * w.bh;
    int base = 0;
    bool listed = true;
    for (int64_t c0 = 0; c0 < nbox; c0 += NT) {
        const int64_t i = c0 + threadIdx.x;
        int x = 0, y = 0;
        bool mem = false;
        if (i < nbox) {
            y = w.y0 + static_cast<int>(i / w.bw);
            x = w.x0 + static_cast<int>(i % w.bw);
            mem = in_window(w, x, y);
        }
        const uint64_t ball = __ballot(mem);
        if (lane == 0) sCnt[wave] = static_cast<uint32_t>(__popcll(ball));
        __syncthreads();
        int off = base, tot = 0;
#pragma unroll
        for (int v = 0; v < NW; ++v) {
            off += v < wave ? static_cast<int>(sCnt[v]) : 0;
            tot += static_cast<int>(sCnt[v]);
        }
        __syncthreads();
        if (mem) {
            const int slot = off + __popcll(ball & ((1ull << lane) - 1ull));
            if (slot < WCAP) {
                const float v = pixel(f, x, y);
                sPos[slot] = static_cast<uint32_t>(x - w.x0) | (static_cast<uint32_t>(y - w.y0) << 16);
                sVal[slot] = v;
                if (c) {
                    const double I = static_cast<double>(v);
                    c[0] += 1.0;
                    c[1] += I;
                    c[2] += I * I;
                }
            }
        }
        base += tot;
        if (base > WCAP) {
            listed = false;
            break;
        }
    }
    __syncthreads();
    Members m;
    m.pos = sPos;
    m.val = sVal;
    m.n = listed ? base : 0;
    m.listed = listed;
    return m;
}

// Calls fn(x, y, I) for every member handled by this thread.
template <class F>
__device__ __forceinline__ void for_members(const RingFrame& f, const Window& w, const Members& M, F&& fn) {
    if (M.listed) {
        for (int i = threadIdx.x; i < M.n; i += NT) {
            const uint32_t p = M.pos[i];
            fn(w.x0 + static_cast<int>(p & 0xffffu), w.y0 + static_cast<int>(p >> 16), static_cast<double>(M.val[i]));
        }
    } else {
        const int64_t nbox = static_cast<int64_t>(w.bw) * w.bh;
        for (int64_t i = threadIdx.x; i < nbox; i += NT) {
            const int y = w.y0 + static_cast<int>(i / w.bw), x = w.x0 + static_cast<int>(i % w.bw);
            if (in_window(w, x, y)) fn(x, y, static_cast<double>(pixel(f, x, y)));
        }
    }
}

struct Prof {
    double g, rho, dgdrho;
};

__device__ __forceinline__ Prof profile(const double* th, double inv2s2, double invs2, int x, int y) {
    Prof p;
    const double dx = x - th[0], dy = y - th[1];
    p.rho = sqrt(dx * dx + dy * dy);
    const double t = p.rho - th[2];
    p.g = exp(-(t * t) * inv2s2);
    p.dgdrho = -p.g * t * invs2;
    return p;
}

// dg/d(cx, cy, r); at rho = 0 the centre derivatives are taken as 0.
__device__ __forceinline__ void profile_grad(const Prof& p, const double* th, int x, int y, double d[3]) {
    const double safe = p.rho > 0.0 ? p.rho : 1.0;
    const double q = p.dgdrho / safe;
    d[0] = -(x - th[0]) * q;
    d[1] = -(y - th[1]) * q;
    d[2] = -p.dgdrho;
}

// Closed-form (A, B) from n, sum g, sum g^2, sum I, sum I g (Cramer's rule on the 2x2 normal
// equations); an empty window gives (0, 0), a singular system A = 0, B = mean I.
__device__ __forceinline__ void solve_ab(double n, double Sg, double Sgg, double SI, double SIg, double& A,
                                         double& B) {
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

// (A, B) at ring th: sums n, g, g^2, I, I g.
__device__ void fit_ab(const RingFrame& f, const Window& w, const Members& M, const double* th, double inv2s2,
                       double invs2, double* sred, double& A, double& B) {
    double s[5] = {0, 0, 0, 0, 0};
    for_members(f, w, M, [&](int x, int y, double I) {
        const Prof p = profile(th, inv2s2, invs2, x, y);
        s[0] += 1.0;
        s[1] += p.g;
        s[2] += p.g * p.g;
        s[3] += I;
        s[4] += I * p.g;
    });
    block_sum<5>(s, sred);
    solve_ab(s[0], s[1], s[2], s[3], s[4], A, B);
}

__global__ __launch_bounds__(NT) void k_fit_loss(RingArgs a, int backward) {
    __shared__ uint32_t sPos[WCAP_LOSS];
    __shared__ float sVal[WCAP_LOSS];
    __shared__ double sred[NW * 5];
    __shared__ uint32_t sCnt[NW];
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
        const Members M = build_members<WCAP_LOSS>(f, w, sPos, sVal, sCnt);
        const double th[3] = {a.theta[3 * j], a.theta[3 * j + 1], a.theta[3 * j + 2]};
        double A, B;
        fit_ab(f, w, M, th, inv2s2, invs2, sred, A, B);
        if (!backward) {
            double s[1] = {0.0};
            for_members(f, w, M, [&](int x, int y, double I) {
                const double e = I - B - A * profile(th, inv2s2, invs2, x, y).g;
                s[0] += e * e;
            });
            block_sum<1>(s, sred);
            if (threadIdx.x == 0) {
                a.loss[j] = s[0];
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
        for_members(f, w, M, [&](int x, int y, double I) {
            const Prof p = profile(th, inv2s2, invs2, x, y);
            const double e = I - B - A * p.g;
            if (a.grad_img)
                atomicAdd(&a.grad_img[f.grad_off + static_cast<int64_t>(y) * f.W + x], static_cast<float>(gl * 2.0 * e));
            double d[3];
            profile_grad(p, th, x, y, d);
            const double c = -2.0 * A * e;
            s[0] += c * d[0];
            s[1] += c * d[1];
            s[2] += c * d[2];
        });
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

// State of an LM step at one ring position, from one sweep.
struct LmPoint {
    double A, B, L;
    double JtJ[6];   // xx, xy, xr, yy, yr, rr
    double mJte[3];  // -J^T e
};

__device__ LmPoint lm_point(const RingFrame& f, const Window& w, const Members& M, const double* th, double n,
                            double SI, double SII, double inv2s2, double invs2, double* sred) {
    // sums: g, g^2, I g, d d^T (6), d I (3), d (3), d g (3)
    double s[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) s[k] = 0.0;
    for_members(f, w, M, [&](int x, int y, double I) {
        const Prof p = profile(th, inv2s2, invs2, x, y);
        double d[3];
        profile_grad(p, th, x, y, d);
        s[0] += p.g;
        s[1] += p.g * p.g;
        s[2] += I * p.g;
        s[3] += d[0] * d[0];
        s[4] += d[0] * d[1];
        s[5] += d[0] * d[2];
        s[6] += d[1] * d[1];
        s[7] += d[1] * d[2];
        s[8] += d[2] * d[2];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            s[9 + k] += d[k] * I;
            s[12 + k] += d[k];
            s[15 + k] += d[k] * p.g;
        }
    });
    block_sum<18>(s, sred);
    LmPoint q;
    solve_ab(n, s[0], s[1], SI, s[2], q.A, q.B);
    q.L = SII - q.A * s[2] - q.B * SI;
    const double A2 = q.A * q.A;
#pragma unroll
    for (int k = 0; k < 6; ++k) q.JtJ[k] = A2 * s[3 + k];
#pragma unroll
    for (int k = 0; k < 3; ++k) q.mJte[k] = q.A * (s[9 + k] - q.B * s[12 + k] - q.A * s[15 + k]);
    return q;
}

__global__ __launch_bounds__(NT) void k_refine(RingArgs a) {
    __shared__ uint32_t sPos[WCAP_REFINE];
    __shared__ float sVal[WCAP_REFINE];
    __shared__ double sred[NW * 18];
    __shared__ uint32_t sCnt[NW];
    const double inv2s2 = 1.0 / (2.0 * a.s * a.s), invs2 = 1.0 / (a.s * a.s);
    for (int64_t j = blockIdx.x; j < a.m; j += gridDim.x) {
        const int fi = a.frame_of ? a.frame_of[j] : 0;
        if (fi < 0 || fi >= a.nframes) {
            if (threadIdx.x == 0) {
                for (int c = 0; c < 3; ++c) a.theta_out[3 * j + c] = __builtin_nan("");
                if (a.loss) a.loss[j] = __builtin_nan("");
                if (a.steps_out) a.steps_out[j] = 0;
            }
            continue;
        }
        const RingFrame f = a.frames[fi];
        const Window w = make_window(a.theta0 + 3 * j, a.halfwidth, f.W, f.H);
        double c[3] = {0, 0, 0};   // n, sum I, sum I^2 over the fixed window
        const Members M = build_members<WCAP_REFINE>(f, w, sPos, sVal, sCnt, c);
        if (!M.listed) {
            c[0] = c[1] = c[2] = 0.0;
            for_members(f, w, M, [&](int, int, double I) {
                c[0] += 1.0;
                c[1] += I;
                c[2] += I * I;
            });
        }
        block_sum<3>(c, sred);
        double th[3] = {a.theta0[3 * j], a.theta0[3 * j + 1], a.theta0[3 * j + 2]};
        double lam = a.lam0;
        LmPoint cur = lm_point(f, w, M, th, c[0], c[1], c[2], inv2s2, invs2, sred);
        int taken = 0;
        // a converged step lowers the limit to itself; the loop has no early exit, which keeps
        // the kernel within 256 registers (2 waves per SIMD)
        int lim = a.iters;
        for (int it = 0; it < lim; ++it) {
            ++taken;
            // (J^T J + lam diag(J^T J)) d = -J^T e, solved redundantly by every thread
            const double* J = cur.JtJ;
            double Mx[3][3] = {{J[0] + lam * J[0], J[1], J[2]},
                               {J[1], J[3] + lam * J[3], J[4]},
                               {J[2], J[4], J[5] + lam * J[5]}};
            double b[3] = {cur.mJte[0], cur.mJte[1], cur.mJte[2]};
            double d[3] = {0, 0, 0};
            if (!solve3(Mx, b, d)) {
                lam *= a.lam_up;
                continue;
            }
            // converged: every component of the update within tol (false for a NaN update).
            // Every thread holds the same sums, so the flag is uniform (read from the first lane)
            if (__builtin_amdgcn_readfirstlane((fabs(d[0]) <= a.tol && fabs(d[1]) <= a.tol && fabs(d[2]) <= a.tol) ? 1 : 0))
                lim = it + 1;
            const double cand[3] = {th[0] + d[0], th[1] + d[1], th[2] + d[2]};
            const LmPoint nxt = lm_point(f, w, M, cand, c[0], c[1], c[2], inv2s2, invs2, sred);
            if (nxt.L < cur.L) {
                th[0] = cand[0];
                th[1] = cand[1];
                th[2] = cand[2];
                cur = nxt;
                lam *= a.lam_down;
            } else {
                lam *= a.lam_up;
            }
        }
        if (threadIdx.x == 0) {
            a.theta_out[3 * j] = th[0];
            a.theta_out[3 * j + 1] = th[1];
            a.theta_out[3 * j + 2] = th[2];
            if (a.loss) a.loss[j] = cur.L;
            if (a.steps_out) a.steps_out[j] = taken;
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
