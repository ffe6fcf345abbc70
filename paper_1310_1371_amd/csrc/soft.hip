// Differentiable extension of the ridge-directed Hough transform: the soft accumulator
// (each ridge pixel splats its curvature weight -k_- bilinearly at p +- r X_- on every
// radius level, X_- the continuous eigenvector), its adjoint, the adjoint of the 2x2
// eigensolve, and the adjoint of the Hessian operator (transposed separable correlations
// with reflect-101 fold-back).  The paper's voting is integer and non-differentiable; this
// path relaxes it over the same ridge set and the same Hessian (Methods, "Algorithm
// implementation"; Results, "Directed ridge detection & votes collection").
//
// Kernels
//   k_hess_gather   Hessian planes -> per-ridge (Ixx, Iyy, Ixy)
//   k_soft_bin      per ridge: eigensolve in fp64, bin by 16x16 pixels (slot arrays)
//   k_soft_fwd      one workgroup per (32x32 tile, 8 levels): gathers the bins whose ridges
//                   can reach the tile at those radii, clips each (ridge, sign) ray to the
//                   tile, splats into LDS with float atomics, writes the tile once
//   k_soft_bwd      one wave per ridge: lanes over levels, both signs, gathers the upstream
//                   gradient at the 4 splat cells, reduces d/dw and d/dX_-, then applies the
//                   eigen adjoint -> d/d(Ixx, Iyy, Ixy)
//   k_scatter       per-ridge Hessian gradients -> three planes
//   k_adj_pass<D>   one transposed 1D correlation with fold-back along x or y
//
// Splat positions are formed in fp64 with separately rounded operations (x + (s r) ux), so
// the cell a splat lands in is decided exactly as a float64 reference decides it.
#include "rd_internal.h"

namespace rd {
namespace {

constexpr int NT = 256;
constexpr int ST = SOFT_TILE;
constexpr int SL = SOFT_LEVELS;
// bins a tile can gather from: rays reach r_max + 2 <= R_LIMIT + 3 pixels beyond the tile
constexpr int SPAN_MAX = (ST + 1 + 2 * (R_LIMIT + 3)) / BIN + 2;
constexpr int CB_MAX = SPAN_MAX * SPAN_MAX;
static_assert(CB_MAX <= 2 * NT, "candidate bins are scanned two per thread");

struct Geo {
    double km, kp, ux, uy, d, scale;
};

// Eigen-decomposition of [[a, b], [b, c]]: k_- = t - d, k_+ = t + d with t = (a + c) / 2,
// h = (a - c) / 2, d = sqrt(h^2 + b^2).  X_- is (-b, h + d) for h >= 0 and
// sign(b) (h - d, b) for h < 0 (sign(0) = +1), normalised: the unit vector (-sin t, cos t),
// t = atan2(2b, a - c) / 2 in (-pi/2, pi/2], without trigonometry or cancellation.
// Isotropic (d = 0): X_- = (0, 1).
__device__ __forceinline__ Geo geometry(double a, double c, double b) {
    Geo g;
    const double t = 0.5 * (a + c);
    const double h = 0.5 * (a - c);
    g.d = sqrt(h * h + b * b);
    g.km = t - g.d;
    g.kp = t + g.d;
    double vx, vy;
    if (g.d == 0.0) {
        vx = 0.0;
        vy = 1.0;
    } else if (h >= 0.0) {
        vx = -b;
        vy = h + g.d;
    } else {
        const double sg = b < 0.0 ? -1.0 : 1.0;
        vx = sg * (h - g.d);
        vy = sg * b;
    }
    const double inv = 1.0 / sqrt(vx * vx + vy * vy);
    g.ux = vx * inv;
    g.uy = vy * inv;
    g.scale = fmax(fmax(fabs(a), fabs(c)), fabs(b));
    return g;
}

// Splat position p + s r u, each operation rounded on its own (no fused multiply-add).
__device__ __forceinline__ double splat_pos(int p, double sr, double u) {
    return __dadd_rn(static_cast<double>(p), __dmul_rn(sr, u));
}

__global__ __launch_bounds__(NT) void k_hess_gather(const double* planes, int W, int H, const int32_t* xy, int64_t n,
                                                    double* hess) {
    const int64_t plane = static_cast<int64_t>(W) * H;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const int x = xy[2 * i], y = xy[2 * i + 1];
        if (x < 0 || x >= W || y < 0 || y >= H) continue;
        const int64_t g = static_cast<int64_t>(y) * W + x;
        hess[3 * i] = planes[g];
        hess[3 * i + 1] = planes[plane + g];
        hess[3 * i + 2] = planes[2 * plane + g];
    }
}

__global__ __launch_bounds__(NT) void k_soft_bin(SoftBinArgs a) {
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * NT) {
        const int x = a.xy[2 * i], y = a.xy[2 * i + 1];
        if (x < 0 || x >= a.W || y < 0 || y >= a.H) {
            atomicOr(a.flags, 2u);
            continue;
        }
        const Geo g = geometry(a.hess[3 * i], a.hess[3 * i + 1], a.hess[3 * i + 2]);
        const int64_t bin = static_cast<int64_t>(y >> BIN_SHIFT) * a.nbx + (x >> BIN_SHIFT);
        const uint32_t slot = atomicAdd(&a.bin_count[bin], 1u);
        if (slot >= static_cast<uint32_t>(BIN_CAP)) {
            atomicOr(a.flags, 1u);
            continue;
        }
        const int64_t o = bin * BIN_CAP + slot;
        a.sxy[o] = static_cast<uint32_t>(x) | (static_cast<uint32_t>(y) << 16);
        a.sux[o] = g.ux;
        a.suy[o] = g.uy;
        a.sw[o] = static_cast<float>(-g.km);
    }
}

// Exclusive block-wide prefix sum of one value per thread; *total receives the sum.
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t* sWave, uint32_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) sWave[wave] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        const uint32_t c = sWave[w];
        base += w < wave ? c : 0u;
        tot += c;
    }
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

// Integer level range (superset) over which o + r d stays in [lo, hi).  Only a superset is
// needed (every splat is bounds-checked), so fp32 with a reciprocal and one level of margin
// on each side serves.
__device__ __forceinline__ void clip_axis(double o, double d, double lo, double hi, int& r0, int& r1) {
    const float df = static_cast<float>(d);
    if (fabsf(df) <= 1e-6f) {                  // moves at most (R_LIMIT + 3) 1e-6 px: keep a margin
        if (o < lo - 1.001 || o > hi + 0.001) {
            r0 = 1;
            r1 = 0;
        }
        return;
    }
    const float inv = __builtin_amdgcn_rcpf(df);
    float t0 = static_cast<float>(lo - o) * inv, t1 = static_cast<float>(hi - o) * inv;
    if (t0 > t1) {
        const float tt = t0;
        t0 = t1;
        t1 = tt;
    }
    t0 = fmaxf(t0, static_cast<float>(r0) - 2.0f);
    t1 = fminf(t1, static_cast<float>(r1) + 2.0f);
    r0 = max(r0, static_cast<int>(ceilf(t0)) - 2);
    r1 = min(r1, static_cast<int>(floorf(t1)) + 2);
}

__global__ __launch_bounds__(NT) void k_soft_fwd(SoftFwdArgs a) {
    __shared__ float sAcc[SL * ST * ST];
    __shared__ uint32_t sBin[CB_MAX];
    __shared__ uint32_t sPre[CB_MAX + 1];
    __shared__ uint32_t sWave[NT / 64];

    const int tid = threadIdx.x;
    const int ntx = (a.W + ST - 1) / ST;
    const int tile = blockIdx.x;
    const int tx0 = (tile % ntx) * ST, ty0 = (tile / ntx) * ST;
    const int ra = a.r_lo + static_cast<int>(blockIdx.y) * SL;
    const int rb = min(ra + SL - 1, a.r_lo + a.L - 1);
    const int nl = rb - ra + 1;

    for (int i = tid; i < nl * ST * ST; i += NT) sAcc[i] = 0.0f;

    // ---- candidate bins: some pixel of the bin at a distance in [ra - 1, rb + 1] from the
    // region [tx0 - 1, tx0 + ST] x [ty0 - 1, ty0 + ST] where a splat can touch the tile
    const int reach = rb + 2;
    const int bx0 = max(0, (tx0 - 1 - reach) >> BIN_SHIFT), bx1 = min(a.nbx - 1, (tx0 + ST + reach) >> BIN_SHIFT);
    const int by0 = max(0, (ty0 - 1 - reach) >> BIN_SHIFT), by1 = min(a.nby - 1, (ty0 + ST + reach) >> BIN_SHIFT);
    const int spanx = bx1 - bx0 + 1, nsq = spanx * (by1 - by0 + 1);
    uint32_t keep[2] = {0, 0}, cnt[2] = {0, 0}, bins[2] = {0, 0};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int i = 2 * tid + k;
        if (i < nsq) {
            const int bx = bx0 + i % spanx, by = by0 + i / spanx;
            const uint32_t bin = static_cast<uint32_t>(by * a.nbx + bx);
            const uint32_t c = min(a.bin_count[bin], static_cast<uint32_t>(BIN_CAP));
            const double px0 = bx * BIN, px1 = bx * BIN + BIN - 1, py0 = by * BIN, py1 = by * BIN + BIN - 1;
            const double qx0 = tx0 - 1, qx1 = tx0 + ST, qy0 = ty0 - 1, qy1 = ty0 + ST;
            const double gx = fmax(0.0, fmax(px0 - qx1, qx0 - px1)), gy = fmax(0.0, fmax(py0 - qy1, qy0 - py1));
            const double mx = fmax(fabs(px1 - qx0), fabs(qx1 - px0)), my = fmax(fabs(py1 - qy0), fabs(qy1 - py0));
            const bool ok = c > 0 && sqrt(gx * gx + gy * gy) <= rb + 1.0 && sqrt(mx * mx + my * my) >= ra - 1.0;
            keep[k] = ok ? 1u : 0u;
            cnt[k] = ok ? c : 0u;
            bins[k] = bin;
        }
    }
    uint32_t nb = 0, nrid = 0;
    const uint32_t pos = block_scan(keep[0] + keep[1], sWave, &nb);
    const uint32_t pre = block_scan(cnt[0] + cnt[1], sWave, &nrid);
    if (keep[0]) {
        sBin[pos] = bins[0];
        sPre[pos] = pre;
    }
    if (keep[1]) {
        sBin[pos + keep[0]] = bins[1];
        sPre[pos + keep[0]] = pre + cnt[0];
    }
    if (tid == 0) sPre[nb] = nrid;
    __syncthreads();

    // ---- splat every ridge, both signs, over the levels whose footprint meets the tile (one
    // lane per ridge: the bin search and the loads are shared by the two signs)
    for (uint32_t ri = tid; ri < nrid; ri += NT) {
        uint32_t lo = 0, hi = nb;          // largest k with sPre[k] <= ri
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (sPre[mid] <= ri) lo = mid;
            else hi = mid;
        }
        const int64_t slot = static_cast<int64_t>(sBin[lo]) * BIN_CAP + (ri - sPre[lo]);
        const uint32_t v = a.sxy[slot];
        const int x = static_cast<int>(v & 0xffffu), y = static_cast<int>(v >> 16);
        const double ux = a.sux[slot], uy = a.suy[slot];
        const double w = static_cast<double>(a.sw[slot]);
        for (int sg = 0; sg < 2; ++sg) {
            const double sgn = sg ? -1.0 : 1.0;
            int r0 = ra, r1 = rb;
            clip_axis(x, sgn * ux, tx0 - 1.0, tx0 + static_cast<double>(ST), r0, r1);
            clip_axis(y, sgn * uy, ty0 - 1.0, ty0 + static_cast<double>(ST), r0, r1);
            for (int r = r0; r <= r1; ++r) {
                const double sr = sgn * r;
                const double px = splat_pos(x, sr, ux), py = splat_pos(y, sr, uy);
                const double fi = floor(px), fj = floor(py);
                const double fx = px - fi, fy = py - fj;
                const int ci = static_cast<int>(fi) - tx0, cj = static_cast<int>(fj) - ty0;
                float* lvl = sAcc + (r - ra) * ST * ST;
#pragma unroll
                for (int dj = 0; dj < 2; ++dj) {
                    const int yy = cj + dj;
                    if (yy < 0 || yy >= ST || ty0 + yy >= a.H) continue;
                    const double by = dj ? fy : 1.0 - fy;
#pragma unroll
                    for (int di = 0; di < 2; ++di) {
                        const int xx = ci + di;
                        if (xx < 0 || xx >= ST || tx0 + xx >= a.W) continue;
                        const double bx = di ? fx : 1.0 - fx;
                        atomicAdd(&lvl[yy * ST + xx], static_cast<float>(w * (bx * by)));
                    }
                }
            }
        }
    }
    __syncthreads();

    const int64_t plane = static_cast<int64_t>(a.W) * a.H;
    float* out = a.acc + static_cast<int64_t>(ra - a.r_lo) * plane;
    for (int i = tid; i < nl * ST * ST; i += NT) {
        const int l = i / (ST * ST), rem = i - l * ST * ST;
        const int yy = rem / ST, xx = rem - yy * ST;
        const int X = tx0 + xx, Y = ty0 + yy;
        if (X < a.W && Y < a.H) out[l * plane + static_cast<int64_t>(Y) * a.W + X] = sAcc[i];
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ __launch_bounds__(NT) void k_soft_bwd(SoftBwdArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t plane = static_cast<int64_t>(a.W) * a.H;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * (NT / 64) + (threadIdx.x >> 6); i < a.n;
         i += static_cast<int64_t>(gridDim.x) * (NT / 64)) {
        const int x = a.xy[2 * i], y = a.xy[2 * i + 1];
        const Geo g = geometry(a.hess[3 * i], a.hess[3 * i + 1], a.hess[3 * i + 2]);
        const double w = -g.km;
        double gw = 0.0, gux = 0.0, guy = 0.0;
        // one lane per level, both signs (2L pairs in one round of 64 lanes up to L = 64)
        for (int li = lane; li < a.L; li += 64)
#pragma unroll
        for (int sg = 0; sg < 2; ++sg) {
            const double sgn = sg ? -1.0 : 1.0;
            const double sr = sgn * (a.r_lo + li);
            const double px = splat_pos(x, sr, g.ux), py = splat_pos(y, sr, g.uy);
            const double fi = floor(px), fj = floor(py);
            const double fx = px - fi, fy = py - fj;
            const int i0 = static_cast<int>(fi), j0 = static_cast<int>(fj);
            const float* G = a.grad_acc + li * plane;
#pragma unroll
            for (int dj = 0; dj < 2; ++dj) {
                const int cj = j0 + dj;
                if (cj < 0 || cj >= a.H) continue;
                const double by = dj ? fy : 1.0 - fy;
#pragma unroll
                for (int di = 0; di < 2; ++di) {
                    const int ci = i0 + di;
                    if (ci < 0 || ci >= a.W) continue;
                    const double bx = di ? fx : 1.0 - fx;
                    const double gv = static_cast<double>(G[static_cast<int64_t>(cj) * a.W + ci]);
                    gw += gv * bx * by;
                    gux += w * gv * (di ? 1.0 : -1.0) * by * sr;
                    guy += w * gv * bx * (dj ? 1.0 : -1.0) * sr;
                }
            }
        }
        gw = wave_sum(gw);
        gux = wave_sum(gux);
        guy = wave_sum(guy);
        if (lane == 0) {
            // dL/dk_- = -gw; dk_- = X_-^T dH X_-; dX_- = (X_+^T dH X_-) / (k_- - k_+) X_+
            const double gk = -gw;
            const double vx = g.uy, vy = -g.ux;
            double dxx = gk * g.ux * g.ux, dyy = gk * g.uy * g.uy, dxy = gk * 2.0 * g.ux * g.uy;
            if (g.d > 1e-12 * g.scale) {
                const double alpha = (gux * vx + guy * vy) / (g.km - g.kp);
                dxx += alpha * vx * g.ux;
                dyy += alpha * vy * g.uy;
                dxy += alpha * (vx * g.uy + vy * g.ux);
            } else if (a.n_iso) {
                atomicAdd(a.n_iso, 1u);
            }
            a.grad_hess[3 * i] = dxx;
            a.grad_hess[3 * i + 1] = dyy;
            a.grad_hess[3 * i + 2] = dxy;
        }
    }
}

__global__ __launch_bounds__(NT) void k_scatter(ScatterArgs a) {
    const int64_t plane = static_cast<int64_t>(a.W) * a.H;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * NT) {
        const int x = a.xy[2 * i], y = a.xy[2 * i + 1];
        if (x < 0 || x >= a.W || y < 0 || y >= a.H) continue;
        const int64_t g = static_cast<int64_t>(y) * a.W + x;
#pragma unroll
        for (int c = 0; c < 3; ++c) atomicAdd(&a.planes[c * plane + g], static_cast<float>(a.grad_hess[3 * i + c]));
    }
}

// out(q) = sum over extended positions e that mirror to q (e = q, -q, 2(n-1) - q within
// [-R, n-1+R]) of sum_j taps[j] in(e - j + R), inputs outside [0, n-1] contributing zero:
// the transpose of out(x) = sum_j taps[j] in(reflect101(x + j - R)).
template <int DIR>
__global__ __launch_bounds__(NT) void k_adj_pass(AdjPassArgs a) {
    const int64_t npx = static_cast<int64_t>(a.W) * a.H;
    const int n = DIR == 0 ? a.W : a.H;
    const int R = a.R;
    for (int64_t idx = blockIdx.x * (int64_t)NT + threadIdx.x; idx < npx; idx += (int64_t)gridDim.x * NT) {
        const int y = static_cast<int>(idx / a.W), x = static_cast<int>(idx - static_cast<int64_t>(y) * a.W);
        const int q = DIR == 0 ? x : y;
        int pre[3];
        int np = 0;
        pre[np++] = q;
        if (q >= 1 && q <= R) pre[np++] = -q;
        if (q <= n - 2 && q >= n - 1 - R) pre[np++] = 2 * (n - 1) - q;
        double tot = 0.0;
        for (int c = 0; c < a.ncomp; ++c) {
            const float* in = a.in[c];
            double acc = 0.0;
            for (int k = 0; k < np; ++k) {
                const int e = pre[k];
                for (int j = 0; j <= 2 * R; ++j) {
                    const int src = e - j + R;
                    if (src < 0 || src >= n) continue;
                    const int64_t o = DIR == 0 ? static_cast<int64_t>(y) * a.W + src : static_cast<int64_t>(src) * a.W + x;
                    acc += a.taps[c][j] * static_cast<double>(in[o]);
                }
            }
            if (a.sum) {
                tot += acc;
            } else {
                const float v = static_cast<float>(a.scale * acc);
                a.out[c][idx] = a.accumulate ? a.out[c][idx] + v : v;
            }
        }
        if (a.sum) {
            const float v = static_cast<float>(a.scale * tot);
            a.out[0][idx] = a.accumulate ? a.out[0][idx] + v : v;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_fill(T* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) p[i] = T(0);
}

int grid_for(int64_t n, int cap) {
    const int64_t b = (n + NT - 1) / NT;
    return static_cast<int>(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace

hipError_t launch_hess_gather(const double* planes, int W, int H, const int32_t* xy, int64_t n, double* hess,
                              hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_hess_gather, dim3(grid_for(n, 4096)), dim3(NT), 0, s, planes, W, H, xy, n, hess);
    return hipGetLastError();
}

hipError_t launch_soft_bin(const SoftBinArgs& a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_soft_bin, dim3(grid_for(a.n, 4096)), dim3(NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_soft_forward(const SoftFwdArgs& a, hipStream_t s) {
    const int tiles = ((a.W + ST - 1) / ST) * ((a.H + ST - 1) / ST);
    const int chunks = (a.L + SL - 1) / SL;
    if (tiles <= 0 || chunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_soft_fwd, dim3(tiles, chunks), dim3(NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_soft_backward(const SoftBwdArgs& a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    const int64_t b = (a.n + NT / 64 - 1) / (NT / 64);
    hipLaunchKernelGGL(k_soft_bwd, dim3(static_cast<int>(b < 65536 ? b : 65536)), dim3(NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_scatter_grad_hess(const ScatterArgs& a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(a.n, 4096)), dim3(NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_adj_pass(const AdjPassArgs& a, int dir, hipStream_t s) {
    const int64_t npx = static_cast<int64_t>(a.W) * a.H;
    if (npx <= 0) return hipSuccess;
    if (dir == 0) hipLaunchKernelGGL(k_adj_pass<0>, dim3(grid_for(npx, 8192)), dim3(NT), 0, s, a);
    else hipLaunchKernelGGL(k_adj_pass<1>, dim3(grid_for(npx, 8192)), dim3(NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(n, 8192)), dim3(NT), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(n, 8192)), dim3(NT), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace rd
