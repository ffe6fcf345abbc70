// Fused pre-processing + ridge kernel (method steps 1-2).
//
// One workgroup owns a TW x TH output tile of a frame and computes, entirely in LDS:
//   load (reflect-101 borders, u16 or f32 -> f32)     input tile + (RG + 3) px halo
//   horizontal Gaussian (fp64)                         rows of the input tile
//   vertical Gaussian (fp64)                           smoothed image G on tile + 3 px
//   5x5 second-order Sobel / 64 and the 2x2 eigensolve k_- (fp64) on tile + 1 px
//   direction code q = rint(2^14 X_-) where k_- < T_k
//   ridge test (k_- < T_k, strict minimum along the nearest lattice direction of X_-)
//   and wave-ballot compaction of the ridge pixels into their 16x16 bins.
// Only the input is read from HBM and only the ridges are written, so nothing of the
// smoothed image, the Hessian or k_- ever goes to memory (except in the dense stage mode,
// which writes k_- and q, and optionally the Hessian planes, of a single frame).
//
// The filters run in fp64 by default: the Hessian is a small difference of large smoothed
// values (e.g. a 12-bit frame with a 600-count background and curvatures of order 1
// count/px^2).  CDNA fp64 FMA issues at the fp32 (non-packed) rate, so fp64 costs no issue
// slots, only registers and LDS.  The fp32 variant (rd_params.curvature_fp32) first takes the
// mean of the loaded tile out of every input pixel: second derivatives are blind to a
// constant, so this changes only the magnitude the filters carry, and with it the rounding.
// It halves the LDS planes and the registers of the filter windows, which lets three
// workgroups share a CU where the fp64 kernel fits two.
//
// Single reflect-101 extension of the raw image is enough for the two-step definition
// (blur with mirrored borders, then Sobel with mirrored borders): with a symmetric
// Gaussian the blurred extension is itself mirror-symmetric about both edges.
#include "rd_internal.h"

namespace rd {
namespace {

// Mirror about the edge pixel (-1 -> 1, n -> n-2).  Positions farther out than one
// reflection only feed outputs outside the frame; they are clamped to stay in bounds.
__device__ __forceinline__ int reflect101(int i, int n) {
    i = i < 0 ? -i : i;
    i = i > n - 1 ? 2 * (n - 1) - i : i;
    return i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
}

template <typename TIN>
__device__ __forceinline__ float load_px(const void* img, int64_t pitch, int x, int y) {
    const TIN* row = reinterpret_cast<const TIN*>(reinterpret_cast<const char*>(img) + (int64_t)y * pitch);
    return static_cast<float>(row[x]);
}

// Direction code of X_- for the eigenvalue t - d of [[t+h, c], [c, t-h]], d = sqrt(h^2+c^2).
// The eigenvector is (-c, h + d) for h >= 0 and (h - d, c) for h < 0 (no cancellation in
// either branch); at an isotropic point (d == 0) X_- = (0, 1).
// Code of the direction of a nonzero vector (vx, vy): rint(2^14 v / |v|) per component, the
// sign chosen so that qy > 0, or qy == 0 and qx > 0.
__device__ __forceinline__ uint32_t vector_code(double vx, double vy) {
    const double inv = 16384.0 / sqrt(vx * vx + vy * vy);
    int qx = static_cast<int>(rint(vx * inv));
    int qy = static_cast<int>(rint(vy * inv));
    if (qy < 0 || (qy == 0 && qx < 0)) {
        qx = -qx;
        qy = -qy;
    }
    return (static_cast<uint32_t>(qx) & 0xffffu) | (static_cast<uint32_t>(qy) << 16);
}

__device__ __forceinline__ uint32_t direction_code(double h, double c, double d) {
    if (d == 0.0) return vector_code(0.0, 1.0);
    return h >= 0.0 ? vector_code(-c, h + d) : vector_code(h - d, c);
}

// Directed edges: the unit gradient's code, (0, 1) where the gradient vanishes.
__device__ __forceinline__ uint32_t gradient_code(double ix, double iy, double g) {
    return g == 0.0 ? vector_code(0.0, 1.0) : vector_code(ix, iy);
}

// Neighbour offset along X_-: nearest of the 8 lattice directions, in integers
// (13573 / 32768 ~ tan(pi / 8)).
__device__ __forceinline__ void nms_offset(uint32_t q, int& nx, int& ny) {
    const int qx = static_cast<int16_t>(q & 0xffffu);
    const int qy = static_cast<int16_t>(q >> 16);
    const int ax = qx < 0 ? -qx : qx;
    const int ay = qy < 0 ? -qy : qy;
    if (13573 * ax > 32768 * ay) {
        nx = 1; ny = 0;
    } else if (13573 * ay > 32768 * ax) {
        nx = 0; ny = 1;
    } else {
        nx = 1; ny = (qx * qy > 0) ? 1 : -1;
    }
}

template <int TW_, int TH_, int RG_, typename TC_>
struct StencilShape {
    using TC = TC_;                                // filter arithmetic: double or float
    static constexpr int TW = TW_, TH = TH_, RG = RG_;
    static constexpr int HALO = RG + 3;            // Gaussian + Sobel + NMS neighbour
    static constexpr int IW = TW + 2 * HALO;       // input tile
    static constexpr int IH = TH + 2 * HALO;
    static constexpr int IWP = IW | 1;             // odd pitch: conflict-free row-per-lane reads
    static constexpr int HC = TW + 6;              // columns of the horizontally smoothed rows
    static constexpr int GH = TH + 6;              // rows of G
    static constexpr int KW = TW + 2, KH = TH + 2; // k_- region (tile + 1 px)
    static constexpr int MH = 10;                  // outputs per thread, horizontal pass
    static constexpr int MV = 13;                  // vertical pass
    static constexpr int MS = 6;                   // Sobel/eigen pass
    static constexpr int NBX = TW / BIN, NBY = TH / BIN;
    static constexpr int SZ_I = IH * IWP * 4;
    static constexpr int SZ_G = GH * HC * (int)sizeof(TC);
    static constexpr int SZ_H = IH * HC * (int)sizeof(TC);
    static constexpr int SZ_K = KH * KW * (int)sizeof(TC);
    static constexpr int SZ_Q = KH * KW * 4;
    static constexpr int SZ_A = SZ_I > SZ_G ? SZ_I : SZ_G;
    static constexpr int SZ_B = SZ_H > (SZ_K + SZ_Q) ? SZ_H : (SZ_K + SZ_Q);
    static constexpr int LDS = SZ_A + SZ_B;
    static_assert(TW % BIN == 0 && TH % BIN == 0, "tiles hold whole bins");
    static_assert(LDS <= 65536, "static LDS limit");
    // workgroups per CU the register allocation plans for: three for the fp32 kernel up to
    // RG = 8 (168 registers, a few spilled; its LDS allows it), else what the registers give
    static constexpr int MINB = (sizeof(TC) == 4 && RG <= 8 && 3 * LDS <= 160 * 1024) ? 3 : 1;
};

constexpr int NT = 256;

template <typename TIN, typename SH, bool DENSE>
__global__ __launch_bounds__(NT, SH::MINB) void k_stencil(StencilArgs a) {
    using TC = typename SH::TC;
    constexpr bool F32 = sizeof(TC) == 4;
    constexpr int TW = SH::TW, TH = SH::TH, RG = SH::RG, HALO = SH::HALO;
    constexpr int IW = SH::IW, IH = SH::IH, IWP = SH::IWP, HC = SH::HC, GH = SH::GH;
    constexpr int KW = SH::KW, KH = SH::KH, MH = SH::MH, MV = SH::MV, MS = SH::MS;
    constexpr int NBX = SH::NBX, NB = SH::NBX * SH::NBY;

    __shared__ __align__(16) uint8_t smem[SH::LDS];
    __shared__ uint32_t wcount[NB][NT / 64];
    // the frame table of a launch of up to FRAMES_LDS frames, read once per workgroup
    __shared__ FrameDesc sFr[FRAMES_LDS];
    __shared__ float sRed[NT / 64];                             // fp32: the tile mean
    float* sI = reinterpret_cast<float*>(smem);                 // region A
    TC* sG = reinterpret_cast<TC*>(smem);                       // region A (after sI dies)
    TC* sH = reinterpret_cast<TC*>(smem + SH::SZ_A);            // region B
    TC* sK = reinterpret_cast<TC*>(smem + SH::SZ_A);            // region B (after sH dies)
    uint32_t* sQ = reinterpret_cast<uint32_t*>(smem + SH::SZ_A + SH::SZ_K);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const TC kthr = static_cast<TC>(a.k_threshold);
    TC gw[RG + 1];                                              // Gaussian taps
#pragma unroll
    for (int i = 0; i <= RG; ++i) gw[i] = static_cast<TC>(a.g[i]);

    const bool fr_lds = a.nframes <= FRAMES_LDS;
    if (fr_lds) {
        for (int i = tid; i < a.nframes; i += NT) sFr[i] = a.frames[i];
        __syncthreads();
    }

    for (int t = blockIdx.x; t < a.total_tiles; t += gridDim.x) {
        // ---- which frame / tile
        int f = 0;                                  // last frame whose first tile is <= t
        for (int hi = a.nframes; hi - f > 1;) {
            const int mid = (f + hi) >> 1;
            if ((fr_lds ? sFr[mid].tile0 : a.frames[mid].tile0) <= t) f = mid; else hi = mid;
        }
        const FrameDesc fd = fr_lds ? sFr[f] : a.frames[f];
        const int W = fd.W, H = fd.H;
        const int tiles_x = (W + TW - 1) / TW;
        const int local = t - fd.tile0;
        const int x0 = (local % tiles_x) * TW;
        const int y0 = (local / tiles_x) * TH;

        // ---- load the input tile with mirrored borders: a thread's loads (up to twenty at a
        // time) are all issued before any of them is stored, so their latencies overlap
        float part = 0.0f;                          // fp32: this thread's share of the tile sum
        {
            constexpr int NLD = (IH * IW + NT - 1) / NT, G = NLD < 20 ? NLD : 20;
#pragma unroll
            for (int k0 = 0; k0 < NLD; k0 += G) {
                float v[G];
#pragma unroll
                for (int k = 0; k < G; ++k) {
                    const int i = tid + (k0 + k) * NT;
                    v[k] = 0.0f;
                    if (k0 + k < NLD && i < IH * IW) {
                        const int r = i / IW, c = i - r * IW;
                        const int gy = reflect101(y0 - HALO + r, H);
                        const int gx = reflect101(x0 - HALO + c, W);
                        v[k] = load_px<TIN>(fd.img, fd.pitch, gx, gy);
                    }
                }
#pragma unroll
                for (int k = 0; k < G; ++k) {
                    const int i = tid + (k0 + k) * NT;
                    if (k0 + k < NLD && i < IH * IW) {
                        const int r = i / IW, c = i - r * IW;
                        sI[r * IWP + c] = v[k];
                        if (F32) part += v[k];
                    }
                }
            }
        }
        if (F32) {
            // the tile mean out of every pixel (any constant would do: it cancels in the
            // second derivatives, up to rounding)
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
            if (lane == 0) sRed[wave] = part;
            __syncthreads();
            const float mean = ((sRed[0] + sRed[1]) + (sRed[2] + sRed[3])) * (1.0f / (IH * IW));
            for (int i = tid; i < IH * IW; i += NT) {
                const int r = i / IW, c = i - r * IW;
                sI[r * IWP + c] -= mean;
            }
        }
        __syncthreads();

        // ---- horizontal Gaussian: sH[r][c] <- image x = x0 - 3 + c, all IH rows
        constexpr int NSH = (HC + MH - 1) / MH;
        for (int task = tid; task < IH * NSH; task += NT) {
            const int r = task % IH, c0 = (task / IH) * MH;
            const float* src = sI + r * IWP + c0;
            TC w[MH + 2 * RG];
#pragma unroll
            for (int i = 0; i < MH + 2 * RG; ++i) w[i] = (c0 + i < IW) ? static_cast<TC>(src[i]) : TC(0);
#pragma unroll
            for (int m = 0; m < MH; ++m) {
                TC acc = gw[0] * w[m + RG];
#pragma unroll
                for (int i = 1; i <= RG; ++i) acc = fma(gw[i], w[m + RG - i] + w[m + RG + i], acc);
                if (c0 + m < HC) sH[r * HC + c0 + m] = acc;
            }
        }
        __syncthreads();

        // ---- vertical Gaussian: sG[r][c] <- image (x0 - 3 + c, y0 - 3 + r)
        constexpr int NSV = (GH + MV - 1) / MV;
        for (int task = tid; task < HC * NSV; task += NT) {
            const int c = task % HC, r0 = (task / HC) * MV;
            TC w[MV + 2 * RG];
#pragma unroll
            for (int i = 0; i < MV + 2 * RG; ++i) w[i] = (r0 + i < IH) ? sH[(r0 + i) * HC + c] : TC(0);
#pragma unroll
            for (int m = 0; m < MV; ++m) {
                TC acc = gw[0] * w[m + RG];
#pragma unroll
                for (int i = 1; i <= RG; ++i) acc = fma(gw[i], w[m + RG - i] + w[m + RG + i], acc);
                if (r0 + m < GH) sG[(r0 + m) * HC + c] = acc;
            }
        }
        __syncthreads();

        // ---- Sobel / 64 and eigensolve: sK[r][c] <- image (x0 - 1 + c, y0 - 1 + r)
        constexpr int NSS = (KH + MS - 1) / MS;
        for (int task = tid; task < KW * NSS; task += NT) {
            const int c = task % KW, r0 = (task / KW) * MS;
            TC d2x[MS + 4], s5x[MS + 4], d1x[MS + 4];
#pragma unroll
            for (int i = 0; i < MS + 4; ++i) {
                const int gr = r0 + i < GH ? r0 + i : GH - 1;
                const TC* g = sG + gr * HC + c;
                const TC gm2 = g[0], gm1 = g[1], g0 = g[2], gp1 = g[3], gp2 = g[4];
                d2x[i] = (gm2 + gp2) - TC(2) * g0;
                s5x[i] = (gm2 + gp2) + TC(4) * (gm1 + gp1) + TC(6) * g0;
                d1x[i] = (gp2 - gm2) + TC(2) * (gp1 - gm1);
            }
#pragma unroll
            for (int m = 0; m < MS; ++m) {
                const int r = r0 + m;
                if (r < KH && a.edge) {
                    // directed edges: Ix = S5_y D1_x G / 128, Iy = D1_y S5_x G / 128, m = -|grad I|
                    const TC ix = ((d1x[m] + d1x[m + 4]) + TC(4) * (d1x[m + 1] + d1x[m + 3]) + TC(6) * d1x[m + 2]) * TC(1.0 / 128.0);
                    const TC iy = ((s5x[m + 4] - s5x[m]) + TC(2) * (s5x[m + 3] - s5x[m + 1])) * TC(1.0 / 128.0);
                    const TC g = sqrt(ix * ix + iy * iy);
                    const TC k = -g;
                    sK[r * KW + c] = k;
                    sQ[r * KW + c] = (DENSE || k < kthr) ? gradient_code(ix, iy, g) : 0u;
                } else if (r < KH) {
                    const TC ixx = ((d2x[m] + d2x[m + 4]) + TC(4) * (d2x[m + 1] + d2x[m + 3]) + TC(6) * d2x[m + 2]) * TC(1.0 / 64.0);
                    const TC iyy = ((s5x[m] + s5x[m + 4]) - TC(2) * s5x[m + 2]) * TC(1.0 / 64.0);
                    const TC ixy = ((d1x[m + 4] - d1x[m]) + TC(2) * (d1x[m + 3] - d1x[m + 1])) * TC(1.0 / 64.0);
                    const TC tr = TC(0.5) * (ixx + iyy);
                    const TC h = TC(0.5) * (ixx - iyy);
                    const TC d = sqrt(h * h + ixy * ixy);
                    const TC k = tr - d;
                    sK[r * KW + c] = k;
                    sQ[r * KW + c] = (DENSE || k < kthr) ? direction_code(h, ixy, d) : 0u;
                    if (DENSE && a.hess_dense && r >= 1 && r <= TH && c >= 1 && c <= TW) {
                        const int x = x0 - 1 + c, y = y0 - 1 + r;
                        if (x < W && y < H) {
                            const int64_t g = (int64_t)y * W + x, plane = (int64_t)W * H;
                            a.hess_dense[g] = ixx;
                            a.hess_dense[plane + g] = iyy;
                            a.hess_dense[2 * plane + g] = ixy;
                        }
                    }
                }
            }
        }
        __syncthreads();

        if (DENSE) {
            // stage mode: k_- and q of the tile interior
            for (int i = tid; i < TW * TH; i += NT) {
                const int py = i / TW, px = i - py * TW;
                const int x = x0 + px, y = y0 + py;
                if (x < W && y < H) {
                    const int o = (py + 1) * KW + px + 1;
                    const int64_t g = (int64_t)y * W + x;
                    if (a.k_dense) a.k_dense[g] = static_cast<float>(sK[o]);
                    if (a.q_dense) {
                        const uint32_t q = sQ[o];
                        a.q_dense[2 * g] = static_cast<int16_t>(q & 0xffffu);
                        a.q_dense[2 * g + 1] = static_cast<int16_t>(q >> 16);
                    }
                }
            }
        } else {
            // ---- ridge test and compaction, one 16x16 bin per 256 threads
            uint64_t masks[NB];
            const int bpx = tid & (BIN - 1), bpy = tid >> BIN_SHIFT;
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int px = (j % NBX) * BIN + bpx, py = (j / NBX) * BIN + bpy;
                const int x = x0 + px, y = y0 + py;
                bool ridge = false;
                if (x >= 1 && x <= W - 2 && y >= 1 && y <= H - 2) {
                    const int o = (py + 1) * KW + px + 1;
                    const TC k = sK[o];
                    if (k < kthr) {
                        int nx, ny;
                        nms_offset(sQ[o], nx, ny);
                        ridge = (k < sK[o + ny * KW + nx]) && (k < sK[o - ny * KW - nx]);
                    }
                }
                masks[j] = __ballot(ridge);
                if (lane == 0) wcount[j][wave] = static_cast<uint32_t>(__popcll(masks[j]));
            }
            __syncthreads();
            const int bx0 = x0 >> BIN_SHIFT, by0 = y0 >> BIN_SHIFT;
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int bx = bx0 + (j % NBX), by = by0 + (j / NBX);
                if (bx >= fd.nbx || by >= fd.nby) continue;
                const int64_t bin = fd.bin0 + (int64_t)by * fd.nbx + bx;
                const uint64_t m = masks[j];
                if ((m >> lane) & 1ull) {
                    uint32_t pos = static_cast<uint32_t>(__popcll(m & ((1ull << lane) - 1ull)));
                    for (int w2 = 0; w2 < wave; ++w2) pos += wcount[j][w2];
                    const int px = (j % NBX) * BIN + bpx, py = (j / NBX) * BIN + bpy;
                    const int o = (py + 1) * KW + px + 1;
                    const int64_t slot = bin * BIN_CAP + pos;
                    a.rxy[slot] = static_cast<uint32_t>(x0 + px) | (static_cast<uint32_t>(y0 + py) << 16);
                    a.rq[slot] = sQ[o];
                    a.rk[slot] = static_cast<float>(sK[o]);
                }
                if (tid == 0) {
                    uint32_t tot = 0;
                    for (int w2 = 0; w2 < NT / 64; ++w2) tot += wcount[j][w2];
                    a.bin_count[bin] = tot;
                }
            }
            if (tid == 0 && a.ridge_total) {     // statistics, striped over 64 counters
                uint32_t tot = 0;
                for (int j = 0; j < NB; ++j)
                    for (int w2 = 0; w2 < NT / 64; ++w2) tot += wcount[j][w2];
                if (tot) atomicAdd(&a.ridge_total[t & 63], static_cast<unsigned long long>(tot));
            }
        }
        __syncthreads();   // LDS is reused by the next tile of a persistent block
    }
}

template <typename TIN, int TW, int TH, int RG, bool DENSE>
hipError_t launch_t(const StencilArgs& a, hipStream_t s) {
    if (a.fp32) {
        hipLaunchKernelGGL((k_stencil<TIN, StencilShape<TW, TH, RG, float>, DENSE>), dim3(a.total_tiles), dim3(NT), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_stencil<TIN, StencilShape<TW, TH, RG, double>, DENSE>), dim3(a.total_tiles), dim3(NT), 0, s, a);
    }
    return hipGetLastError();
}

template <typename TIN, int RG>
hipError_t launch_shape(const StencilArgs& a, int variant, bool dense, hipStream_t s) {
    if (dense) return launch_t<TIN, 64, (RG <= 8 ? 32 : 16), RG, true>(a, s);   // stage output
    switch (variant) {
        case 1: return launch_t<TIN, 32, 32, RG, false>(a, s);
        case 2: return launch_t<TIN, 64, 16, RG, false>(a, s);
        default: return launch_t<TIN, 64, (RG <= 8 ? 32 : 16), RG, false>(a, s);
    }
}

template <typename TIN>
hipError_t launch_rg(const StencilArgs& a, int rg, int variant, bool dense, hipStream_t s) {
    if (rg <= 4) return launch_shape<TIN, 4>(a, variant, dense, s);
    if (rg <= 8) return launch_shape<TIN, 8>(a, variant, dense, s);
    if (rg <= 12) return launch_shape<TIN, 12>(a, variant, dense, s);
    return launch_shape<TIN, 16>(a, variant, dense, s);
}

}  // namespace

void stencil_tile_dims(int variant, int rg, bool dense, int* tw, int* th) {
    if (dense || variant == 0) {
        *tw = 64;
        *th = rg <= 8 ? 32 : 16;
    } else if (variant == 1) {
        *tw = 32;
        *th = 32;
    } else {
        *tw = 64;
        *th = 16;
    }
}

hipError_t launch_stencil(const StencilArgs& a, int dtype, int rg, int variant, bool dense, hipStream_t s) {
    if (a.total_tiles <= 0) return hipSuccess;
    if (dtype == RD_U16) return launch_rg<uint16_t>(a, rg, variant, dense, s);
    return launch_rg<float>(a, rg, variant, dense, s);
}

}  // namespace rd
