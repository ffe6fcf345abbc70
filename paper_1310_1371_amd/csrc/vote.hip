// Directed voting, radius-dependent smoothing, 1/r normalisation and 3x3x3 peak search
// (method steps 3-4), fused in one LDS-resident kernel.
//
// A workgroup owns a T x T spatial tile and a chunk of consecutive radius levels
// [rc0, rc1) in which it searches for peaks.  It needs the raw accumulator of levels
// rc0 - 1 .. rc1 on the tile grown by 1 px (the 3x3x3 box) plus the smoothing half-width
// K, so it:
//   1. zeroes a u16 histogram for those levels in LDS (two counters per 32-bit word);
//   2. gathers, from the 16x16 ridge bins whose pixels can reach the region at those
//      radii, every ridge pixel and adds its +/- votes with LDS atomics (exact integers,
//      the direction is the fixed-point code, offset floor((r q + 2^13) / 2^14));
//   3. per level: compacts the hotspots (A > T_int) of the tile + 1 px, evaluates the
//      integer score S_int = sum W(|dx|) W(|dy|) A with 15-bit weight factors (one window
//      row per thread, merged with LDS 64-bit atomics), keeps scores above the level's
//      integer threshold in a 3-level rotating map, and runs the 3x3x3 comparison for the
//      previous level (scores at different levels compare as S_int / r, exactly, by
//      cross-multiplication; a plateau keeps its first voxel in (r, y, x) order).
// The dense accumulator volume never exists in memory: this is the GPU form of the
// paper's rotating three-level sub-spaces with hotspot-only processing.
//
// A neighbour whose score is at or below the threshold can never beat a candidate, which
// is above it, so keeping only above-threshold scores leaves every decision unchanged.
#include "rd_internal.h"

namespace rd {
namespace {

constexpr int NT = 256;
constexpr int NW = NT / 64;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t n = __shfl_up(v, o, 64);
        if (lane >= o) v += n;
    }
    return v;
}

// Exclusive prefix over the block; *total receives the sum.  Contains __syncthreads.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* s_wave, uint32_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan(v, lane);
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        if (w < wave) base += s_wave[w];
        tot += s_wave[w];
    }
    *total = tot;
    return base + inc - v;
}

__device__ __forceinline__ uint32_t get_u16(const uint32_t* s, int idx) {
    return (s[idx >> 1] >> ((idx & 1) << 4)) & 0xffffu;
}

template <int T, bool DUMP>
__global__ __launch_bounds__(NT) void k_vote(VoteArgs a) {
    constexpr int SR = T + 2;
    extern __shared__ __align__(16) uint32_t sA[];
    __shared__ uint64_t sS[3 * SR * SR];
    __shared__ uint16_t sHot[SR * SR];
    __shared__ uint32_t sBin[NT];
    __shared__ uint32_t sPre[NT + 1];
    __shared__ uint32_t sWave[NW];
    __shared__ uint32_t sCnt;
    __shared__ uint32_t sWf[K_MAX + 1];

    const int tid = threadIdx.x, lane = tid & 63;
    const int n_items = a.total_vtiles * a.nchunks;

    for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int t = item / a.nchunks;
        const int chunk = item - t * a.nchunks;
        int f = 0;
        while (f + 1 < a.nframes && a.frames[f + 1].vtile0 <= t) ++f;
        const FrameDesc fd = a.frames[f];
        const int W = fd.W, H = fd.H;
        const int tiles_x = (W + T - 1) / T;
        const int local = t - fd.vtile0;
        const int x0 = (local % tiles_x) * T, y0 = (local / tiles_x) * T;

        const int rc0 = a.chunk_start[chunk], rc1 = a.chunk_start[chunk + 1];
        const int l0 = rc0 - 1, l1 = rc1;           // accumulator levels, inclusive
        const int Kc = a.ktab[l1 - a.lbase];        // widest window of the chunk
        // score region (tile + 1 px) and accumulator region (+ K), clipped to the frame
        const int sx0 = max(x0 - 1, 0), sx1 = min(x0 + T + 1, W);
        const int sy0 = max(y0 - 1, 0), sy1 = min(y0 + T + 1, H);
        const int ax0 = max(sx0 - Kc, 0), ax1 = min(sx1 + Kc, W);
        const int ay0 = max(sy0 - Kc, 0), ay1 = min(sy1 + Kc, H);
        const int AW = ax1 - ax0, AH = ay1 - ay0;
        const int AWP = (AW + 1) & ~1;
        const int plane = AWP * AH;                 // u16 per level, even
        const int nlev = l1 - l0 + 1;

        for (int i = tid; i < (nlev * plane) >> 1; i += NT) sA[i] = 0u;
        __syncthreads();

        // ---- gather the ridges of every bin that can reach the region, and vote
        const int reach = l1 + 1;
        const int bxlo = max((ax0 - reach) >> BIN_SHIFT, 0);
        const int bxhi = min((ax1 - 1 + reach) >> BIN_SHIFT, fd.nbx - 1);
        const int bylo = max((ay0 - reach) >> BIN_SHIFT, 0);
        const int byhi = min((ay1 - 1 + reach) >> BIN_SHIFT, fd.nby - 1);
        const int nbxr = bxhi - bxlo + 1;
        const int ncand = nbxr * (byhi - bylo + 1);
        const int far_lo = max(l0 - 1, 0);
        for (int cb = 0; cb < ncand; cb += NT) {
            const int i = cb + tid;
            uint32_t cnt = 0;
            int64_t bin = 0;
            if (i < ncand) {
                const int bx = bxlo + i % nbxr, by = bylo + i / nbxr;
                bin = fd.bin0 + (int64_t)by * fd.nbx + bx;
                // pixel-box distances between the bin and the accumulator region
                const int px0 = bx << BIN_SHIFT, px1 = px0 + BIN - 1;
                const int py0 = by << BIN_SHIFT, py1 = py0 + BIN - 1;
                const int gx = max(0, max(ax0 - px1, px0 - (ax1 - 1)));
                const int gy = max(0, max(ay0 - py1, py0 - (ay1 - 1)));
                const int fx = max(abs(px0 - (ax1 - 1)), abs(px1 - ax0));
                const int fy = max(abs(py0 - (ay1 - 1)), abs(py1 - ay0));
                const bool keep = gx * gx + gy * gy <= reach * reach && fx * fx + fy * fy >= far_lo * far_lo;
                if (keep) cnt = min(a.bin_count[bin], static_cast<uint32_t>(BIN_CAP));
            }
            uint32_t total;
            const uint32_t pre = block_excl_scan(cnt, sWave, &total);
            sBin[tid] = static_cast<uint32_t>(bin - fd.bin0);
            sPre[tid] = pre;
            if (tid == 0) sPre[NT] = total;
            __syncthreads();
            for (uint32_t j = tid; j < total; j += NT) {
                int lo = 0, hi = NT;            // largest lo with sPre[lo] <= j
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (sPre[mid] <= j) lo = mid; else hi = mid;
                }
                const int64_t slot = (fd.bin0 + sBin[lo]) * BIN_CAP + (j - sPre[lo]);
                const uint32_t xy = a.rxy[slot], q = a.rq[slot];
                const int x = xy & 0xffffu, y = xy >> 16;
                const int qx = static_cast<int16_t>(q & 0xffffu), qy = static_cast<int16_t>(q >> 16);
                for (int l = l0; l <= l1; ++l) {
                    const int ox = (l * qx + 8192) >> 14, oy = (l * qy + 8192) >> 14;
                    const int base = (l - l0) * plane;
                    int u = x + ox - ax0, v = y + oy - ay0;
                    if (static_cast<unsigned>(u) < static_cast<unsigned>(AW) && static_cast<unsigned>(v) < static_cast<unsigned>(AH)) {
                        const int idx = base + v * AWP + u;
                        atomicAdd(&sA[idx >> 1], 1u << ((idx & 1) << 4));
                    }
                    u = x - ox - ax0;
                    v = y - oy - ay0;
                    if (static_cast<unsigned>(u) < static_cast<unsigned>(AW) && static_cast<unsigned>(v) < static_cast<unsigned>(AH)) {
                        const int idx = base + v * AWP + u;
                        atomicAdd(&sA[idx >> 1], 1u << ((idx & 1) << 4));
                    }
                }
            }
            __syncthreads();
        }

        if (DUMP) {
            const int ix1 = min(x0 + T, W), iy1 = min(y0 + T, H);
            const int iw = ix1 - x0, ih = iy1 - y0;
            for (int i = tid; i < nlev * iw * ih; i += NT) {
                const int li = i / (iw * ih), rem = i - li * (iw * ih);
                const int y = y0 + rem / iw, x = x0 + rem % iw;
                a.acc_dump[((int64_t)(l0 + li - a.lbase) * H + y) * W + x] =
                    get_u16(sA, li * plane + (y - ay0) * AWP + (x - ax0));
            }
        }

        // ---- per level: hotspot scores, threshold, and the 3x3x3 search one level behind
        const int SW = sx1 - sx0, SHh = sy1 - sy0;
        for (int l = l0; l <= l1; ++l) {
            const int li = l - l0;
            uint64_t* Sm = sS + (li % 3) * SR * SR;
            const int lg = l - a.lbase;
            for (int i = tid; i < SR * SR; i += NT) Sm[i] = 0ull;
            if (tid == 0) sCnt = 0;
            if (tid <= K_MAX) sWf[tid] = a.wtab[lg * (K_MAX + 1) + tid];
            __syncthreads();
            const uint32_t tint = static_cast<uint32_t>(a.vote_threshold);
            for (int i0 = 0; i0 < SW * SHh; i0 += NT) {
                const int i = i0 + tid;
                bool hot = false;
                int sidx = 0;
                if (i < SW * SHh) {
                    const int vx = sx0 + i % SW, vy = sy0 + i / SW;
                    hot = get_u16(sA, li * plane + (vy - ay0) * AWP + (vx - ax0)) > tint;
                    sidx = (vy - (y0 - 1)) * SR + (vx - (x0 - 1));
                }
                const uint64_t m = __ballot(hot);
                uint32_t base = 0;
                if (lane == 0 && m) base = atomicAdd(&sCnt, static_cast<uint32_t>(__popcll(m)));
                base = __shfl(base, 0, 64);
                if (hot) sHot[base + __popcll(m & ((1ull << lane) - 1ull))] = static_cast<uint16_t>(sidx);
            }
            __syncthreads();
            const int nh = static_cast<int>(sCnt);
            const int K = a.ktab[lg];
            const uint32_t* wf = sWf;
            const int rows = 2 * K + 1;
            for (int task = tid; task < nh * rows; task += NT) {
                const int h = task / rows, dy = task - h * rows - K;
                const int sidx = sHot[h];
                const int vx = x0 - 1 + sidx % SR, vy = y0 - 1 + sidx / SR;
                const int yy = vy + dy;
                if (yy < ay0 || yy >= ay1) continue;
                const int xs = max(vx - K, ax0), xe = min(vx + K, ax1 - 1);
                const int rowbase = li * plane + (yy - ay0) * AWP - ax0;
                uint32_t rs = 0;
                for (int x = xs; x <= xe; ++x) rs += wf[abs(x - vx)] * get_u16(sA, rowbase + x);
                if (rs) atomicAdd(reinterpret_cast<unsigned long long*>(&Sm[sidx]),
                                  static_cast<unsigned long long>(wf[abs(dy)]) * rs);
            }
            __syncthreads();
            const uint64_t thr = a.thr[lg];
            for (int h = tid; h < nh; h += NT) {
                const int sidx = sHot[h];
                const uint64_t s = Sm[sidx];
                if (DUMP && a.score_dump) {
                    const int vx = x0 - 1 + sidx % SR, vy = y0 - 1 + sidx / SR;
                    if (vx >= x0 && vx < x0 + T && vy >= y0 && vy < y0 + T)
                        a.score_dump[((int64_t)lg * H + vy) * W + vx] = s;
                }
                if (s <= thr) Sm[sidx] = 0ull;
            }
            __syncthreads();
            if (l - 1 >= rc0) {
                const int lm = l - 1;
                const uint64_t* Sp = sS + ((li + 1) % 3) * SR * SR;   // level l - 2
                const uint64_t* Sc = sS + ((li + 2) % 3) * SR * SR;   // level l - 1
                const uint64_t* Sn = Sm;                               // level l
                for (int i = tid; i < T * T; i += NT) {
                    const int iy = i / T, ix = i - iy * T;
                    const int x = x0 + ix, y = y0 + iy;
                    if (x >= W || y >= H) continue;
                    const int o = (iy + 1) * SR + ix + 1;
                    const uint64_t sv = Sc[o];
                    if (!sv) continue;
                    bool peak = true;
#pragma unroll
                    for (int dl = -1; dl <= 1; ++dl) {
                        const uint64_t* Sl = dl < 0 ? Sp : (dl == 0 ? Sc : Sn);
                        const uint64_t ru = static_cast<uint64_t>(lm + dl);
#pragma unroll
                        for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
                            for (int dx = -1; dx <= 1; ++dx) {
                                if (dl == 0 && dy == 0 && dx == 0) continue;
                                const uint64_t su = Sl[o + dy * SR + dx];
                                if (!su) continue;
                                const uint64_t lhs = sv * ru, rhs = su * static_cast<uint64_t>(lm);
                                const bool earlier = dl < 0 || (dl == 0 && (dy < 0 || (dy == 0 && dx < 0)));
                                if (earlier ? !(lhs > rhs) : !(lhs >= rhs)) peak = false;
                            }
                        }
                    }
                    if (peak) {
                        const uint32_t idx = atomicAdd(&a.peak_count[f], 1u);
                        if (idx < static_cast<uint32_t>(a.max_peaks)) {
                            Peak pk;
                            pk.a = x; pk.b = y; pk.r = lm; pk.frame = f; pk.s = sv;
                            a.peaks[fd.peak0 + idx] = pk;
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Scatter a caller-given ridge list into the per-bin slots.
__global__ __launch_bounds__(NT) void k_bin(BinArgs a) {
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * NT) {
        const int x = a.xy[2 * i], y = a.xy[2 * i + 1];
        if (x < 0 || x >= a.W || y < 0 || y >= a.H) {
            atomicOr(a.overflow, 2u);
            continue;
        }
        const int64_t bin = (int64_t)(y >> BIN_SHIFT) * a.nbx + (x >> BIN_SHIFT);
        const uint32_t pos = atomicAdd(&a.bin_count[bin], 1u);
        if (pos >= static_cast<uint32_t>(BIN_CAP)) {
            atomicOr(a.overflow, 1u);
            continue;
        }
        const int64_t slot = bin * BIN_CAP + pos;
        a.rxy[slot] = static_cast<uint32_t>(x) | (static_cast<uint32_t>(y) << 16);
        a.rq[slot] = (static_cast<uint32_t>(static_cast<uint16_t>(a.q[2 * i]))) |
                     (static_cast<uint32_t>(static_cast<uint16_t>(a.q[2 * i + 1])) << 16);
        a.rk[slot] = 0.0f;
    }
}

// Copy the binned ridges of a single frame into caller arrays at per-bin offsets.
__global__ __launch_bounds__(NT) void k_gather(const uint32_t* rxy, const uint32_t* rq, const float* rk,
                                               const uint32_t* bin_count, const int64_t* offsets, int64_t nbins,
                                               int32_t* xy, int16_t* q, float* k) {
    for (int64_t b = blockIdx.x; b < nbins; b += gridDim.x) {
        const uint32_t cnt = bin_count[b];
        for (uint32_t i = threadIdx.x; i < cnt; i += NT) {
            const int64_t src = b * BIN_CAP + i, dst = offsets[b] + i;
            const uint32_t v = rxy[src], w = rq[src];
            if (xy) {
                xy[2 * dst] = static_cast<int32_t>(v & 0xffffu);
                xy[2 * dst + 1] = static_cast<int32_t>(v >> 16);
            }
            if (q) {
                q[2 * dst] = static_cast<int16_t>(w & 0xffffu);
                q[2 * dst + 1] = static_cast<int16_t>(w >> 16);
            }
            if (k) k[dst] = rk[src];
        }
    }
}

}  // namespace

hipError_t launch_gather(const uint32_t* rxy, const uint32_t* rq, const float* rk, const uint32_t* bin_count,
                         const int64_t* offsets, int64_t nbins, int32_t* xy, int16_t* q, float* k, hipStream_t s) {
    const int blocks = static_cast<int>(nbins < 8192 ? nbins : 8192);
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(blocks), dim3(NT), 0, s, rxy, rq, rk, bin_count, offsets, nbins, xy, q, k);
    return hipGetLastError();
}

size_t vote_lds_bytes(int tile, int nlev_max, int kmax) {
    const int side = tile + 2 + 2 * kmax;
    const size_t plane = (size_t)((side + 1) & ~1) * side;
    return ((nlev_max * plane * 2 + 15) / 16) * 16;
}

static bool g_attr_set[2] = {false, false};

hipError_t launch_vote(const VoteArgs& a, size_t lds, bool dump, hipStream_t s) {
    const int items = a.total_vtiles * a.nchunks;
    if (items <= 0) return hipSuccess;
    if (dump) {
        if (!g_attr_set[1]) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_vote<VOTE_TILE, true>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
            if (e != hipSuccess) return e;
            g_attr_set[1] = true;
        }
        hipLaunchKernelGGL((k_vote<VOTE_TILE, true>), dim3(items), dim3(NT), lds, s, a);
    } else {
        if (!g_attr_set[0]) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_vote<VOTE_TILE, false>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
            if (e != hipSuccess) return e;
            g_attr_set[0] = true;
        }
        hipLaunchKernelGGL((k_vote<VOTE_TILE, false>), dim3(items), dim3(NT), lds, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_bin(const BinArgs& a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    int64_t blocks = (a.n + NT - 1) / NT;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_bin, dim3(static_cast<unsigned>(blocks)), dim3(NT), 0, s, a);
    return hipGetLastError();
}

}  // namespace rd
