// Directed voting, radius-dependent smoothing, 1/r normalisation and 3x3x3 peak search
// (method steps 3-4), fused in one LDS-resident kernel.
//
// One persistent workgroup per CU takes T x T spatial tiles from a queue.  For each tile it
// stages, once, the ridge records of the 16x16 bins whose pixels can vote into the tile's
// widest accumulator region, with each sign's level range clipped to that region, and orders
// the (ridge, sign) items that can reach the tile by first level.  It then walks the level
// chunks; a chunk of peak levels [rc0, rc1) needs the raw accumulator of levels rc0 - 1 .. rc1
// on the tile grown by 1 px (the 3x3x3 box) plus the smoothing half-width K.  The chunks are
// cut per tile to fill the LDS histogram, and a chunk's two top levels are the next chunk's
// two bottom ones: their strong voxels (step 4) pass to the next chunk, which then holds and
// votes only its new levels.  Per chunk it:
//   1. clears a u16 histogram of those levels in LDS (two counters per 32-bit word);
//   2. adds every item's votes over its level range with LDS atomics (exact integers: the
//      direction is the fixed-point code, offset floor((r q + 2^13) / 2^14));
//   3. lists the hotspots (A > T_int) of the tile + 1 px as they arise: the atomic returns
//      the counter's old value, and the vote that lifts it past T_int lists the voxel;
//   4. evaluates the integer score S_int = sum W(|dx|) W(|dy|) A of each hotspot with 15-bit
//      weight factors, in tasks of one 8-column band of the window and part of its rows, and
//      keeps the scores above the level's integer threshold in a "strong" list;
//   5. tests each strong voxel of the peak levels against the strong voxels of its 3x3x3 box
//      (scores at different levels compare as S_int / r, exactly, by cross-multiplication; a
//      plateau keeps its first voxel in (r, y, x) order).
// The dense accumulator volume never exists in memory: this is the GPU form of the paper's
// rotating three-level sub-spaces with hotspot-only processing.
//
// A neighbour whose score is at or below the threshold can never beat a candidate, which
// is above it, so comparing against the strong voxels only leaves every decision unchanged.
#include "rd_internal.h"

namespace rd {
namespace {

constexpr int NT = 1024;
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

// floor(x / d) by a multiply-high with m = floor((2^32 - 1) / d) + 1, exact while x * d < 2^32
// (m wraps to 0 for d = 1, which takes x itself)
__device__ __forceinline__ uint32_t div_mulhi(uint32_t x, uint32_t d, uint32_t m) {
    return d == 1u ? x : __umulhi(x, m);
}

__device__ __forceinline__ uint32_t get_u16(const uint32_t* s, int idx) {
    return (s[idx >> 1] >> ((idx & 1) << 4)) & 0xffffu;
}

constexpr int LMAX = R_LIMIT + 3;          // levels r_min - 1 .. r_max + 1 at most
constexpr int NLEV_MAX = VOTE_NLEV_MAX;    // accumulator levels per level chunk
constexpr int ACAP = 1536;                 // staged ridges (with a sign that can reach the tile)
constexpr int PCAP = 160;                  // pieces of the candidate list (rounds of NT candidates)
constexpr int SCAP = 512;                  // above-threshold ("strong") voxels per chunk
constexpr int WC = K_MAX + 8;              // centre tap of the padded weight row
constexpr int NWW = WC + 4;                // u16 pairs per weight row: taps 0 .. 2 WC + 7
constexpr int NS_HASH = 64;                // longer strong lists are tested through a hash table
constexpr int HT = 2048;                   // its slots (u32), in the histogram's storage (free by then)
static_assert(HT * 4 <= VOTE_TABLE_BYTES, "the launch gives the histogram at least the table's size");
constexpr int KEY_BITS = 11;               // score-region index bits of a table key
static_assert(SCAP <= 0xffff && (NLEV_MAX - 1) < (1 << (16 - KEY_BITS)),
              "table entries pack a 16-bit voxel key and a 16-bit index");

// slot of a voxel key (level << KEY_BITS | index in the score region) in the strong-voxel table
__device__ __forceinline__ uint32_t strong_slot(uint32_t key) { return (key * 2654435761u) >> (32 - 11); }

typedef unsigned short ushort2_t __attribute__((ext_vector_type(2)));

// sum of two u16 x u16 products, accumulated in u32 (v_dot2_u32_u16)
__device__ __forceinline__ uint32_t dot2_u16(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_udot2(__builtin_bit_cast(ushort2_t, a), __builtin_bit_cast(ushort2_t, b), c, false);
}

// One block per CU walks the vote tiles of the launch.  For each tile it stages the ridge
// records of every bin that can reach the tile at any radius in LDS once, then runs the
// level chunks over them.
template <int T, bool DUMP, bool PHASES = false>
__global__ __launch_bounds__(NT) void k_vote(VoteArgs a) {
    constexpr int SR = T + 2, SR2 = SR * SR;
    // the hotspot list holds a whole score region (the per-level fallback lists one level's)
    constexpr int HCAP = (SR2 + 255) / 256 * 256;
    static_assert(HT * 4 <= HCAP * 12, "or the table lives in the hotspot list's storage");
    static_assert(SR2 <= (1 << KEY_BITS), "a score-region index fits its part of the table key");
    constexpr int BINS_PER_SIDE = ((T + 2 + 2 * K_MAX + 2 * (R_LIMIT + 2)) >> BIN_SHIFT) + 2;
    static_assert(BINS_PER_SIDE * BINS_PER_SIDE <= NT, "one thread per candidate bin");
    extern __shared__ __align__(16) uint32_t sA[];           // u16 histogram, two per word
    __shared__ uint32_t sRidXY[ACAP];
    __shared__ uint32_t sRidQ[ACAP];
    __shared__ uint32_t sRidR[ACAP];                         // level ranges of both signs (u8 pairs)
    __shared__ uint16_t sOrd[2 * ACAP];                      // (ridge, sign) items by first level
    __shared__ int32_t sCur[PCAP + 1];                       // first candidate round of each piece
    __shared__ int32_t sVt0[FRAMES_LDS];                     // first vote tile of each frame
    __shared__ int32_t sNPieces;
    __shared__ uint32_t sKey[256];                           // counting-sort offsets
    __shared__ uint32_t sNact;                               // items with a non-empty level range
    // hotspot list and scores
    __shared__ __align__(16) uint8_t sScratch[HCAP * 12];
    uint32_t* const sHot = reinterpret_cast<uint32_t*>(sScratch);                        // (level << 16) | index
    unsigned long long* const sHS = reinterpret_cast<unsigned long long*>(sScratch + HCAP * 4);

    __shared__ unsigned long long sStrongS[SCAP];
    __shared__ uint32_t sStrongId[SCAP];
    __shared__ uint8_t sBad[SCAP];                           // strong voxel beaten by a neighbour
    __shared__ __align__(8) uint32_t sBinPre[NT + 1];
    __shared__ uint32_t sBinId[NT];
    // strong voxels handed from a chunk to the next (its two top levels are the next chunk's
    // two bottom levels): in the candidate-bin tables, which a tile staged in one piece does
    // not read after its first chunk's staging
    static_assert(SCAP * 8 <= (NT + 1) * 4 && SCAP <= NT, "the carried list fits the bin tables");
    unsigned long long* const sCarryS = reinterpret_cast<unsigned long long*>(sBinPre);
    uint32_t* const sCarryId = sBinId;
    __shared__ uint16_t sWt[LMAX][K_MAX + 1];                // 15-bit weight factors
    // per chunk level: weights W(|o - WC|) of taps o = 0 .. 2 WC + 8 (zero beyond K), as u16
    // pairs starting at even (sWpE) and odd (sWpO) taps, for two-tap dot products
    __shared__ uint32_t sWpE[NLEV_MAX][NWW];
    __shared__ uint32_t sWpO[NLEV_MAX][NWW];
    __shared__ int sTile, sFrame;
    __shared__ unsigned long long sThr[LMAX];
    __shared__ int32_t sKt[LMAX];
    __shared__ uint32_t sWave[NW];
    __shared__ uint32_t sNh, sNs, sGat;
    __shared__ uint32_t sLevN[NLEV_MAX];                      // strong voxels per chunk level

    const int tid = threadIdx.x, lane = tid & 63;
    const int L = a.nlevels;
    // phase clocks (the profiling instance only): thread 0 reads the shader clock after the
    // barrier that ends each phase, so each span is the workgroup's
    unsigned long long ph_acc[PH_COUNT] = {}, ph_last = 0, ph_start = 0;
    int ph_tiles = 0, ph_tile = -1;
    if (PHASES && tid == 0) ph_start = ph_last = __builtin_readcyclecounter();
    auto stamp = [&](int ph) {
        if (PHASES && tid == 0) {
            const unsigned long long now = __builtin_readcyclecounter();
            ph_acc[ph] += now - ph_last;
            ph_last = now;
        }
    };
    for (int i = tid; i < L * (K_MAX + 1); i += NT) {
        const int li = i / (K_MAX + 1), d = i - li * (K_MAX + 1);
        sWt[li][d] = static_cast<uint16_t>(a.wtab[i]);
    }
    for (int i = tid; i < L; i += NT) {
        sThr[i] = a.thr[i];
        sKt[i] = a.ktab[i];
    }
    if (a.nframes <= FRAMES_LDS)
        for (int i = tid; i < a.nframes; i += NT) sVt0[i] = a.frames[i].vtile0;
    __syncthreads();

    // level i (0 .. L - 1) has radius rbase + rstep i; the chunk table holds level indices and
    // the peak levels are 1 .. L - 2
    const int rbase = a.lbase, rstep = a.r_step;
    auto radius = [&](int i) { return rbase + rstep * i; };
    const float inv_step = 1.0f / static_cast<float>(rstep);   // exact for rstep = 1
    const int i_hi = L - 1;                                    // the top level
    const uint32_t tint = static_cast<uint32_t>(a.vote_threshold);
    uint32_t st_votes = 0;                                              // statistics
    unsigned long long st_hot = 0, st_strong = 0, st_taps = 0;

    for (;;) {
        // tiles are taken from a queue: their cost varies with the number of hotspots
        if (tid == 0) {
            int tq = static_cast<int>(atomicAdd(a.tile_counter, 1u));
            const int qpos = tq;
            if (a.tile_order && tq < a.total_vtiles) tq = static_cast<int>(a.tile_order[tq]);   // costliest first
            if (PHASES && a.tile_clocks) {         // the previous tile's end, this one's start
                const unsigned long long now = __builtin_readcyclecounter();
                if (ph_tile >= 0) a.tile_clocks[4 * ph_tile + 3] = now;
                ph_tile = tq < a.total_vtiles ? tq : -1;
                if (ph_tile >= 0) {
                    a.tile_clocks[4 * tq] = blockIdx.x;
                    a.tile_clocks[4 * tq + 1] = static_cast<unsigned long long>(qpos);
                    a.tile_clocks[4 * tq + 2] = now;
                }
            }
            int fq = 0;                             // last frame whose first vote tile is <= tq
            for (int hi = a.nframes; hi - fq > 1;) {
                const int mid = (fq + hi) >> 1;
                if ((a.nframes <= FRAMES_LDS ? sVt0[mid] : a.frames[mid].vtile0) <= tq) fq = mid; else hi = mid;
            }
            sTile = tq;
            sFrame = fq;
        }
        __syncthreads();
        const int t = sTile;
        if (t >= a.total_vtiles) break;
        const int f = sFrame;
        const FrameDesc fd = a.frames[f];
        const int W = fd.W, H = fd.H;
        const int tiles_x = (W + T - 1) / T;
        const int local = t - fd.vtile0;
        const int x0 = (local % tiles_x) * T, y0 = (local / tiles_x) * T;
        const int sx0 = max(x0 - 1, 0), sx1 = min(x0 + T + 1, W);
        const int sy0 = max(y0 - 1, 0), sy1 = min(y0 + T + 1, H);

        // ---- candidate bins: every bin whose pixels can vote into the tile's widest
        // accumulator region at some level radius
        const int Km = sKt[i_hi];
        const int ux0 = max(sx0 - Km, 0), ux1 = min(sx1 + Km, W);
        const int uy0 = max(sy0 - Km, 0), uy1 = min(sy1 + Km, H);
        const int reach = radius(i_hi) + 1, far_lo = max(rbase - 1, 0);
        const int bxlo = max((ux0 - reach) >> BIN_SHIFT, 0), bxhi = min((ux1 - 1 + reach) >> BIN_SHIFT, fd.nbx - 1);
        const int bylo = max((uy0 - reach) >> BIN_SHIFT, 0), byhi = min((uy1 - 1 + reach) >> BIN_SHIFT, fd.nby - 1);
        const int nbxr = bxhi - bxlo + 1;
        const int ncand = nbxr * (byhi - bylo + 1);
        // at most (T + 2 + 2 K_MAX + 2 (R_LIMIT + 2)) / 16 + 2 = 23 bins per side (< NT in all)
        uint32_t cnt = 0, bin_local = 0;
        if (tid < ncand) {
            const int by = bylo + tid / nbxr, bx = bxlo + (tid - (tid / nbxr) * nbxr);
            const int px0 = bx << BIN_SHIFT, px1 = px0 + BIN - 1;
            const int py0 = by << BIN_SHIFT, py1 = py0 + BIN - 1;
            const int gx = max(0, max(ux0 - px1, px0 - (ux1 - 1)));
            const int gy = max(0, max(uy0 - py1, py0 - (uy1 - 1)));
            const int fx = max(abs(px0 - (ux1 - 1)), abs(px1 - ux0));
            const int fy = max(abs(py0 - (uy1 - 1)), abs(py1 - uy0));
            if (gx * gx + gy * gy <= reach * reach && fx * fx + fy * fy >= far_lo * far_lo) {
                bin_local = static_cast<uint32_t>(by * fd.nbx + bx);
                cnt = min(a.bin_count[fd.bin0 + bin_local], static_cast<uint32_t>(BIN_CAP));
            }
        }
        uint32_t total;
        const uint32_t pre = block_excl_scan(cnt, sWave, &total);
        sBinPre[tid] = pre;
        sBinId[tid] = bin_local;
        if (tid == 0) {
            sBinPre[NT] = total;
            sCur[0] = 0;
            sNPieces = PCAP + 1;                          // known once the first chunk has staged
        }
        const int nrounds = static_cast<int>((total + NT - 1) / NT);

        // Level chunks are cut per tile: a chunk of peak levels [c0, c1) needs the accumulator
        // planes of levels c0 - 1 .. c1 on the tile grown by 1 + K(c1) px (clipped to the
        // frame), except the two bottom ones when the previous chunk handed over their strong
        // voxels (skip = 2).  The chunk takes the most peak levels whose planes fit the
        // launch's histogram storage, at least one (which always fits: the launch holds any
        // one-level chunk of an unclipped tile, and K grows with the level).
        auto plane_u16 = [&](int K) {
            const int AW = min(sx1 + K, W) - max(sx0 - K, 0), AH = min(sy1 + K, H) - max(sy0 - K, 0);
            return ((AW + 8) & ~7) * AH;
        };
        auto chunk_end = [&](int c0, int skip) {
            // lane i tests the end c0 + 2 + i (accumulator levels c0 - 1 .. c0 + 2 + i); the
            // sizes grow with i, so the chunk ends before the first lane that fails
            const int e = c0 + 2 + lane, nl = e - c0 + 2;
            const bool fits = e <= L - 1 && nl <= NLEV_MAX && 2 * (nl - skip) * plane_u16(sKt[e]) <= a.hist_bytes;
            return c0 + 1 + __builtin_ctzll(~__ballot(fits));   // lane NLEV_MAX - 3 fails
        };
        // clear a chunk's histogram, fill its weight rows and empty its hotspot list; the first
        // chunk's here, the next one's during a chunk's 3x3x3 phase, which touches none of these.
        // A chunk that takes over the strong voxels of its two bottom levels (skip = 2) has no
        // planes for them: plane i of the storage holds local level i + skip.
        auto prepare = [&](int c0, int c1, int skip) {
            const int l0 = c0 - 1, l1 = c1;
            const int nlev = l1 - l0 + 1;
            const int words = ((nlev - skip) * plane_u16(sKt[l1])) >> 1;   // whole uint4s
            uint4* a4 = reinterpret_cast<uint4*>(sA);
            const uint4 z = make_uint4(0u, 0u, 0u, 0u);
            for (int i = tid; i < (words >> 2); i += NT) a4[i] = z;
            for (int i = (words & ~3) + tid; i < words; i += NT) sA[i] = 0u;
            for (int i = tid; i < nlev * NWW; i += NT) {
                const int li = i / NWW, j = i - li * NWW;
                const int lg = l0 + li, K = sKt[lg];
                uint32_t wl[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const int o = 2 * j + k, d = o > WC ? o - WC : WC - o;
                    wl[k] = d <= K ? static_cast<uint32_t>(sWt[lg][d]) : 0u;
                }
                sWpE[li][j] = wl[0] | (wl[1] << 16);
                sWpO[li][j] = wl[1] | (wl[2] << 16);
            }
            if (tid == 0) sNh = 0;
        };
        bool carry = false;                                   // strong voxels handed to the next chunk
        int rc0 = 1, rc1 = chunk_end(1, 0);                   // the chunk's peak levels [rc0, rc1)
        prepare(rc0, rc1, 0);
        __syncthreads();
        stamp(PH_SETUP);
        if (PHASES) ++ph_tiles;

        for (bool first_chunk = true;; first_chunk = false) {
            // local levels below `skip` were scored by the previous chunk, which handed over
            // their ncar strong voxels (the scores of a level do not depend on the chunk: its
            // window lies inside every chunk's accumulator region that holds the level).  They
            // join the hotspot list with their scores while the votes run.
            const int skip = carry ? 2 : 0, ncar = carry ? static_cast<int>(sGat) : 0;
            carry = false;
            for (int i = tid; i < ncar; i += NT) {
                const uint32_t h = atomicAdd(&sNh, 1u);
                if (h < static_cast<uint32_t>(HCAP)) {
                    sHot[h] = sCarryId[i];
                    sHS[h] = sCarryS[i];
                }
            }
            const int l0 = rc0 - 1, l1 = rc1;                // accumulator level indices, inclusive
            const int nlev = l1 - l0 + 1;
            const int Kc = sKt[l1];                           // widest window of the chunk
            const int ax0 = max(sx0 - Kc, 0), ax1 = min(sx1 + Kc, W);
            const int ay0 = max(sy0 - Kc, 0), ay1 = min(sy1 + Kc, H);
            const int AW = ax1 - ax0, AH = ay1 - ay0;
            const int AWP = (AW + 8) & ~7;                    // 16-byte rows, >= 1 zero column
            const int plane = AWP * AH;                       // u16 per level, multiple of 8
            // the score region (tile + 1 px) in histogram coordinates
            const int hu0 = sx0 - ax0, hw = sx1 - sx0, hv0 = sy0 - ay0, hh = sy1 - sy0;
            if (tid == 0) sNs = 0;                            // last read by the previous 3x3x3 phase
            if (tid < NLEV_MAX) sLevN[tid] = 0u;
            // ---- votes of the staged ridges.  Only ridges with a sign that can reach the tile
            // are staged.  They are staged once per tile when they fit (ACAP); otherwise the
            // first chunk cuts the candidate list into pieces of whole rounds of NT candidates
            // that fit, and every chunk restages the pieces one after another.
            for (int pc = 0;; ++pc) {
                if (first_chunk || sNPieces > 1) {
                    const int rend = first_chunk ? nrounds : sCur[pc + 1];
                    uint32_t pn = 0;
                    int rd = sCur[pc];
                    for (; rd < rend; ++rd) {
                        const uint32_t g = static_cast<uint32_t>(rd) * NT + tid;
                        uint32_t xy = 0, q = 0, rr = 0x00ff00ffu;   // both signs empty
                        if (g < total) {
                            int lo = 0, hi = NT;                  // largest lo with sBinPre[lo] <= g
                            while (hi - lo > 1) {
                                const int mid = (lo + hi) >> 1;
                                if (sBinPre[mid] <= g) lo = mid; else hi = mid;
                            }
                            const int64_t slot = (fd.bin0 + sBinId[lo]) * BIN_CAP + (g - sBinPre[lo]);
                            xy = a.rxy[slot];
                            q = a.rq[slot];
                            // levels (indices) at which each sign's vote can land in the
                            // tile's widest accumulator region: |rho - l q / 2^14| <= 1/2 per axis
                            const int x = xy & 0xffffu, y = xy >> 16;
                            const int qx = static_cast<int16_t>(q & 0xffffu), qy = static_cast<int16_t>(q >> 16);
                            rr = 0;
#pragma unroll
                            for (int sg = 0; sg < 2; ++sg) {
                                const int sqx = sg ? -qx : qx, sqy = sg ? -qy : qy;
                                // radii first, then level indices with one level of margin
                                float lo_l = static_cast<float>(rbase), hi_l = static_cast<float>(radius(i_hi));
                                bool ok = true;
                                if (sqx != 0) {
                                    const float inv = 16384.0f * __builtin_amdgcn_rcpf(static_cast<float>(sqx));
                                    float e0 = (static_cast<float>(ux0 - x) - 0.5f) * inv;
                                    float e1 = (static_cast<float>(ux1 - 1 - x) + 0.5f) * inv;
                                    if (sqx < 0) { const float tt = e0; e0 = e1; e1 = tt; }
                                    lo_l = fmaxf(lo_l, e0);
                                    hi_l = fminf(hi_l, e1);
                                } else {
                                    ok = x >= ux0 && x < ux1;
                                }
                                if (sqy != 0) {
                                    const float inv = 16384.0f * __builtin_amdgcn_rcpf(static_cast<float>(sqy));
                                    float e0 = (static_cast<float>(uy0 - y) - 0.5f) * inv;
                                    float e1 = (static_cast<float>(uy1 - 1 - y) + 0.5f) * inv;
                                    if (sqy < 0) { const float tt = e0; e0 = e1; e1 = tt; }
                                    lo_l = fmaxf(lo_l, e0);
                                    hi_l = fminf(hi_l, e1);
                                } else {
                                    ok = ok && y >= uy0 && y < uy1;
                                }
                                int la = 255, lb = 0;                      // empty
                                if (ok && lo_l <= hi_l + 2.0f * static_cast<float>(rstep)) {
                                    la = max(0, static_cast<int>(floorf((lo_l - static_cast<float>(rbase)) * inv_step)) - 1);
                                    lb = min(i_hi, static_cast<int>(ceilf((hi_l - static_cast<float>(rbase)) * inv_step)) + 1);
                                    if (lb < la) { la = 255; lb = 0; }
                                }
                                rr |= (static_cast<uint32_t>(la) | (static_cast<uint32_t>(lb) << 8)) << (16 * sg);
                            }
                        }
                        const uint32_t act = ((rr & 0xffu) != 255u || ((rr >> 16) & 0xffu) != 255u) ? 1u : 0u;
                        uint32_t tot;
                        const uint32_t off = block_excl_scan(act, sWave, &tot);
                        if (pn + tot > static_cast<uint32_t>(ACAP)) break;   // first chunk only: the piece ends
                        if (act) {
                            sRidXY[pn + off] = xy;
                            sRidQ[pn + off] = q;
                            sRidR[pn + off] = rr;
                        }
                        pn += tot;
                        __syncthreads();                          // sWave is rewritten next round
                    }
                    if (first_chunk && tid == 0) {
                        sCur[pc + 1] = rd;
                        if (rd >= nrounds) {
                            sNPieces = pc + 1;
                        } else if (pc + 1 == PCAP) {                  // cannot happen: rounds <= 133
                            sNPieces = PCAP;
                            atomicOr(a.error, 1u);
                        }
                    }
                    for (int i = tid; i < 256; i += NT) sKey[i] = 0u;
                    __syncthreads();
                    stamp(PH_STAGE);
                    // order the (ridge, sign) items whose range meets the tile by first level
                    // (counting sort): the lanes of a wave then run level loops of similar
                    // extent; the items that miss the tile (key 255, most of them) are dropped
                    for (int it = tid; it < static_cast<int>(2 * pn); it += NT) {
                        const uint32_t key = (sRidR[it >> 1] >> (16 * (it & 1))) & 0xffu;
                        if (key != 255u) atomicAdd(&sKey[key], 1u);   // empty items are not placed
                    }
                    __syncthreads();
                    if (tid < 64) {
                        uint32_t k4[4];
                        uint32_t sum = 0;
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            k4[e] = sKey[4 * tid + e];
                            sum += k4[e];
                        }
                        const uint32_t inc = wave_incl_scan(sum, lane);
                        uint32_t run = inc - sum;
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            sKey[4 * tid + e] = run;
                            if (4 * tid + e == 255) sNact = run;
                            run += k4[e];
                        }
                    }
                    __syncthreads();
                    for (int it = tid; it < static_cast<int>(2 * pn); it += NT) {
                        const uint32_t key = (sRidR[it >> 1] >> (16 * (it & 1))) & 0xffu;
                        if (key != 255u) sOrd[atomicAdd(&sKey[key], 1u)] = static_cast<uint16_t>(it);
                    }
                    __syncthreads();
                    stamp(PH_SORT);
                }
                // votes: each staged (ridge, sign) item over its level range clipped to this
                // chunk, split between two lanes, or four or eight while the items that start
                // by this chunk's top level (the sorted prefix up to the end of that key's
                // bucket) still fit one pass of the workgroup; the region test below rejects
                // the votes that land in the tile's widest region but outside this chunk's
                const int nc = static_cast<int>(min(sKey[l1], sNact));
                int vsh = 1;
                while (vsh < 3 && (nc << (vsh + 1)) <= NT) ++vsh;
                for (int k = tid; k < (nc << vsh); k += NT) {
                    const int it = sOrd[k >> vsh];
                    const int jr = it >> 1, sg = it & 1;
                    const uint32_t rr = sRidR[jr] >> (16 * sg);
                    const int la0 = max(static_cast<int>(rr & 0xffu), l0 + skip);
                    const int n = min(static_cast<int>((rr >> 8) & 0xffu), l1) - la0 + 1;
                    if (n <= 0) continue;
                    const int part = k & ((1 << vsh) - 1);
                    const int la = la0 + ((part * n) >> vsh), lb = la0 + (((part + 1) * n) >> vsh) - 1;
                    if (la > lb) continue;
                    const uint32_t xy = sRidXY[jr], q = sRidQ[jr];
                    const int x = (xy & 0xffffu) - ax0, y = (xy >> 16) - ay0;
                    const int qx = static_cast<int16_t>(q & 0xffffu), qy = static_cast<int16_t>(q >> 16);
                    // fixed-point offsets, advanced by rstep q per level.  The mirrored vote is
                    // x - floor((r q + 2^13) / 2^14) (not x + rho(r, -q): they differ at exact
                    // halves), which equals x + floor((-r q + 2^13 - 1) / 2^14), so both signs
                    // take the same form with a signed step and rounding constant
                    const int sqx = sg ? -qx : qx, sqy = sg ? -qy : qy;
                    const int rnd = sg ? 8191 : 8192;
                    int accx = radius(la) * sqx + rnd, accy = radius(la) * sqy + rnd;
                    const int stx = rstep * sqx, sty = rstep * sqy;
                    // byte offsets of the u16 counters: 2 u within a row, row stride 2 AWP
                    const int x2 = 2 * x, AW2 = 2 * AW, AWP2 = 2 * AWP;
                    int base = 2 * (la - l0 - skip) * plane;
                    // the vote that lifts a counter past T_int lists the voxel as a hotspot, once,
                    // if it lies in the score region (the tile grown by 1 px).  The slot is taken
                    // at one level step and written at the next, so the wait for the slot comes
                    // with the wait for the next vote instead of adding to the step.
                    uint32_t pend_h = 0xffffffffu, pend_e = 0;
                    // a per-lane address (always sNh): one atomic per listing lane, whose return
                    // is read at the next step (a wave-wide combined atomic is read at once)
                    int zoff = 0;
                    asm volatile("" : "+v"(zoff));
                    uint32_t* const nh_ptr = &sNh + zoff;
                    for (int l = la; l <= lb; ++l) {
                        const int u2 = x2 + 2 * (accx >> 14);
                        const int v = y + (accy >> 14);
                        if (static_cast<unsigned>(u2) < static_cast<unsigned>(AW2) &&
                            static_cast<unsigned>(v) < static_cast<unsigned>(AH)) {
                            const int b = base + static_cast<int>(__umul24(v, AWP2)) + u2;   // 0 <= v < AH
                            const int sh = (b & 2) << 3;
                            const uint32_t old = (atomicAdd(&sA[b >> 2], 1u << sh) >> sh) & 0xffffu;
                            ++st_votes;
                            if (pend_h < static_cast<uint32_t>(HCAP)) {
                                sHot[pend_h] = pend_e;
                                sHS[pend_h] = 0ull;
                            }
                            pend_h = 0xffffffffu;
                            const int u = u2 >> 1;
                            if (old == tint && static_cast<unsigned>(u - hu0) < static_cast<unsigned>(hw) &&
                                static_cast<unsigned>(v - hv0) < static_cast<unsigned>(hh)) {
                                pend_h = atomicAdd(nh_ptr, 1u);
                                pend_e = (static_cast<uint32_t>(l - l0) << 16) |
                                         static_cast<uint32_t>((v - hv0 + sy0 - (y0 - 1)) * SR + (u - hu0 + sx0 - (x0 - 1)));
                            }
                        }
                        accx += stx;
                        accy += sty;
                        base += 2 * plane;
                    }
                    if (pend_h < static_cast<uint32_t>(HCAP)) {
                        sHot[pend_h] = pend_e;
                        sHS[pend_h] = 0ull;
                    }
                }
                __syncthreads();
                stamp(PH_VOTE);
                if (pc + 1 >= sNPieces) break;
            }
            if (tid == 0) sGat = 0;                           // read before the votes' barrier

            const int SHh = sy1 - sy0;

            if (DUMP) {
                const int ix1 = min(x0 + T, W), iy1 = min(y0 + T, H);
                const int iw = ix1 - x0, ih = iy1 - y0;
                for (int li = 0; li < nlev; ++li)
                    for (int i = tid; i < iw * ih; i += NT) {
                        const int y = y0 + i / iw, x = x0 + i % iw;
                        a.acc_dump[((int64_t)(l0 + li) * H + y) * W + x] =
                            get_u16(sA, li * plane + (y - ay0) * AWP + (x - ax0));
                    }
            }

            // ---- integer scores of the hotspots, then the strong (above-threshold) ones
            const uint32_t nh_all = sNh;
            const bool per_level = nh_all > static_cast<uint32_t>(HCAP);
            const int nbm = ((2 * Kc + 7) >> 3) + 1;          // 8-column bands a window can span
            const int npass = per_level ? nlev : 1;
            // The scoring passes, then the 3x3x3 comparison of the strong voxels of the peak levels
            // [rc0, rc1).  When the chunk has more strong voxels than the list holds (the centres
            // of several large rings in one tile), the peak levels are taken in windows
            // [wlo, whi) whose strong voxels at levels wlo - 1 .. whi fit: round 0 scores every
            // hotspot and counts the strong voxels per level; each later round lists a window's
            // strong voxels again, from the hotspot list, or, when the hotspots were listed
            // level by level, by scoring the window's levels again from the histogram.  A window
            // of one peak level that does not fit is an overflow.
            bool windows = false;
            auto strong_in = [&](int lo, int hi) {            // strong voxels at levels lo .. hi
                uint32_t n = 0;
                for (int li = max(lo, 0); li <= min(hi, nlev - 1); ++li) n += sLevN[li];
                return n;
            };
            for (int wlo = 1, round = 0; wlo <= nlev - 2; ++round) {
                int whi = nlev - 1;                            // one window: every peak level
                int p0 = 0, p1 = npass - 1;                    // scoring passes of this round
                if (round > 0) {
                    whi = wlo + 1;
                    if (strong_in(wlo - 1, whi) > static_cast<uint32_t>(SCAP)) {
                        if (tid == 0) atomicOr(a.error, 1u);
                    } else {
                        while (whi <= nlev - 2 && strong_in(wlo - 1, whi + 1) <= static_cast<uint32_t>(SCAP)) ++whi;
                    }
                    __syncthreads();                           // the previous window is done with the list
                    if (tid == 0) sNs = 0;
                    __syncthreads();
                    p0 = 1;
                    p1 = 0;
                    if (per_level) {
                        p0 = wlo - 1;
                        p1 = whi;
                    } else {
                        for (int h = tid; h < static_cast<int>(min(sNh, static_cast<uint32_t>(HCAP))); h += NT) {
                            const uint32_t e = sHot[h];
                            const int li = e >> 16;
                            if (li < wlo - 1 || li > whi) continue;
                            const unsigned long long sc = sHS[h];
                            if (sc > sThr[l0 + li]) {
                                const uint32_t j = atomicAdd(&sNs, 1u);
                                if (j < static_cast<uint32_t>(SCAP)) {
                                    sStrongS[j] = sc;
                                    sStrongId[j] = e;
                                    sBad[j] = 0;
                                }
                            }
                        }
                    }
                }
                const bool first = round == 0;
                for (int pass = p0; pass <= p1; ++pass) {
                if (per_level) {
                    // rare: more hotspots than the list holds; enumerate one level at a time
                    __syncthreads();
                    if (tid == 0) sNh = 0;
                    __syncthreads();
                    const int SW = sx1 - sx0;
                    if (pass < skip) {                        // a carried level: its strong voxels
                        for (int i = tid; i < ncar; i += NT) {
                            const uint32_t e = sCarryId[i];
                            if (static_cast<int>(e >> 16) == pass) {
                                const uint32_t h = atomicAdd(&sNh, 1u);
                                sHot[h] = e;
                                sHS[h] = sCarryS[i];
                            }
                        }
                    } else {
                        for (int i = tid; i < SW * SHh; i += NT) {
                            const int vy = sy0 + i / SW, vx = sx0 + i % SW;
                            if (get_u16(sA, (pass - skip) * plane + (vy - ay0) * AWP + (vx - ax0)) > tint) {
                                const uint32_t h = atomicAdd(&sNh, 1u);
                                sHot[h] = (static_cast<uint32_t>(pass) << 16) |
                                          static_cast<uint32_t>((vy - (y0 - 1)) * SR + (vx - (x0 - 1)));
                                sHS[h] = 0ull;
                            }
                        }
                    }
                    __syncthreads();
                }
                const int nh = static_cast<int>(min(sNh, static_cast<uint32_t>(HCAP)));
                // one task per hotspot, 8-column band of its window (16-byte aligned in the row)
                // and part of the window's row distances: the band's eight horizontal weights
                // stay in registers while the task walks its rows with one 16-byte load each.
                // The distances go in two parts, or in four or eight while the tasks still fit
                // one pass of the workgroup (a short list then waits on shorter row walks).
                int psh = 1;
                while (psh < 3 && (nh * nbm << (psh + 1)) <= NT) ++psh;
                const int ntk = nbm << psh;
                const uint32_t mB = 0xffffffffu / static_cast<uint32_t>(ntk) + 1u;
                for (int task = tid; task < nh * ntk; task += NT) {
                    const int h = static_cast<int>(div_mulhi(static_cast<uint32_t>(task), ntk, mB));
                    const int sub = task - h * ntk, bi = sub >> psh, part = sub & ((1 << psh) - 1);
                    const uint32_t e = sHot[h];
                    const int li = e >> 16, sidx = e & 0xffff;
                    if (li < skip) continue;                       // carried with its score
                    const int lg = l0 + li;
                    const int K = sKt[lg];
                    const int vx = x0 - 1 + sidx % SR, vy = y0 - 1 + sidx / SR;
                    const int cs = max(vx - K, ax0) - ax0, ce = min(vx + K, ax1 - 1) - ax0;
                    const int c0 = ((cs >> 3) + bi) << 3;          // band start, relative to ax0
                    if (c0 > ce) continue;
                    // taps of the band: columns c0 .. c0 + 7 meet weights W(|ax0 + c - vx|), zero
                    // outside the window; columns past the region's right edge are zero padding
                    const int o = ax0 + c0 - vx + WC;               // WC - K - 7 >= 1, o + 7 < 2 WC
                    const uint32_t* wp = (o & 1) ? &sWpO[li][o >> 1] : &sWpE[li][o >> 1];
                    const uint32_t w0 = wp[0], w1 = wp[1], w2 = wp[2], w3 = wp[3];
                    // rows vy - d and vy + d share the weight W(d): part p of the 2^psh takes
                    // d = floor(p (K + 1) / 2^psh) .. floor((p + 1) (K + 1) / 2^psh) - 1 (the
                    // parts cover 0 .. K once; some are empty for small K), rows clipped to the
                    // region, and weights the sum of a pair's two bands once.  A counter takes at most one vote per
                    // lattice offset the rounded r X_- can reach (1016 at r = 127, the largest
                    // level), so two 8-tap bands of weights <= 2^15 stay below 2^31 and the
                    // 32-bit sum is exact.
                    const int dlo = (part * (K + 1)) >> psh, dhi = (((part + 1) * (K + 1)) >> psh) - 1;
                    const int up_max = vy - ay0, dn_max = ay1 - 1 - vy;   // farthest rows in the region
                    const int rstep = AWP >> 3;
                    const uint4* rowc = reinterpret_cast<const uint4*>(sA) + (((li - skip) * plane + (vy - ay0) * AWP + c0) >> 3);
                    const uint16_t* wv = &sWt[lg][0];
                    unsigned long long acc = 0;
                    auto band = [&](const uint4 q) {
                        uint32_t rs = dot2_u16(q.x, w0, 0u);
                        rs = dot2_u16(q.y, w1, rs);
                        rs = dot2_u16(q.z, w2, rs);
                        return dot2_u16(q.w, w3, rs);
                    };
                    // a row outside the region is read at the nearest row inside (the first and
                    // last rows always are) and its band replaced by zero
                    auto row_up = [&](int dd) {
                        const uint32_t b = band(rowc[-min(dd, up_max) * rstep]);
                        return dd <= up_max ? b : 0u;
                    };
                    auto row_dn = [&](int dd) {
                        const uint32_t b = band(rowc[min(dd, dn_max) * rstep]);
                        return (dd > 0 && dd <= dn_max) ? b : 0u;
                    };
                    int d = dlo;
                    for (; d + 1 <= dhi; d += 2) {             // two pairs, four row loads in flight
                        const uint32_t s0 = row_up(d) + row_dn(d), s1 = row_up(d + 1) + row_dn(d + 1);
                        acc += static_cast<unsigned long long>(wv[d]) * s0;
                        acc += static_cast<unsigned long long>(wv[d + 1]) * s1;
                    }
                    if (d <= dhi) acc += static_cast<unsigned long long>(wv[d]) * (row_up(d) + row_dn(d));
                    st_taps += 8 * (max(min(dhi, up_max) - dlo + 1, 0) + max(min(dhi, dn_max) - max(dlo, 1) + 1, 0));
                    if (acc) atomicAdd(&sHS[h], acc);
                }
                __syncthreads();
                stamp(PH_SCORE);
                for (int h = tid; h < nh; h += NT) {
                    const uint32_t e = sHot[h];
                    const int li = e >> 16, sidx = e & 0xffff;
                    const unsigned long long sc = sHS[h];
                    if (DUMP && first && a.score_dump) {
                        const int vx = x0 - 1 + sidx % SR, vy = y0 - 1 + sidx / SR;
                        if (vx >= x0 && vx < x0 + T && vy >= y0 && vy < y0 + T)
                            a.score_dump[((int64_t)(l0 + li) * H + vy) * W + vx] = sc;
                    }
                    if (sc > sThr[l0 + li]) {
                        if (first) atomicAdd(&sLevN[li], 1u);
                        const uint32_t j = atomicAdd(&sNs, 1u);
                        if (j < static_cast<uint32_t>(SCAP)) {
                            sStrongS[j] = sc;
                            sStrongId[j] = e;
                            sBad[j] = 0;
                        }
                    }
                }
                }
                __syncthreads();
                stamp(PH_STRONG);
                if (first) {
                    const uint32_t ns_all = sNs;
                    if (tid == 0) {
                        st_hot += nh_all - ncar;
                        st_strong += static_cast<unsigned long long>(ns_all - ncar);
                    }
                    windows = ns_all > static_cast<uint32_t>(SCAP);
                    // the next chunk's two bottom levels are this chunk's two top levels: hand
                    // their strong voxels over (all of them are in the list unless it overflowed)
                    if (!DUMP && !windows && rc1 <= L - 2 && sNPieces == 1) {
                        for (int j = tid; j < static_cast<int>(ns_all); j += NT) {
                            const uint32_t e = sStrongId[j];
                            if (static_cast<int>(e >> 16) >= nlev - 2) {
                                const uint32_t k = atomicAdd(&sGat, 1u);       // < SCAP
                                sCarryId[k] = e - (static_cast<uint32_t>(nlev - 2) << 16);
                                sCarryS[k] = sStrongS[j];
                            }
                        }
                        carry = true;                          // counted after the next barrier
                    }
                    if (windows) continue;                     // round 1 takes the first window
                }
                const bool in_hist = windows && !per_level;
                const int ns = static_cast<int>(min(sNs, static_cast<uint32_t>(SCAP)));
                // a voxel is tested if its level is a peak level of this window and it lies in the tile
                auto candidate = [&](int j, int& li, int& lm, int& sxr, int& syr) {
                    const uint32_t e = sStrongId[j];
                    li = e >> 16;
                    lm = l0 + li;
                    const int sidx = e & 0xffff;
                    sxr = sidx % SR;
                    syr = sidx / SR;
                    return li >= wlo && li < whi && sxr >= 1 && sxr <= T && syr >= 1 && syr <= T &&
                           x0 - 1 + sxr < W && y0 - 1 + syr < H;
                };
                auto emit = [&](int j, int lm, int sxr, int syr) {
                    const uint32_t idx = atomicAdd(&a.peak_count[f], 1u);
                    if (idx < static_cast<uint32_t>(a.max_peaks)) {
                        Peak pk;
                        pk.a = x0 - 1 + sxr; pk.b = y0 - 1 + syr; pk.r = radius(lm); pk.frame = f; pk.s = sStrongS[j];
                        a.peaks[fd.peak0 + idx] = pk;
                    }
                };
                // a neighbour beats v if its S_int / r is larger, or equal and it comes before v in
                // (r, y, x) order; a neighbour below the threshold cannot, so only strong ones count
                auto beats = [&](unsigned long long sv, int lm, int k, int dl, int dy, int dx) {
                    const unsigned long long lhs = sv * static_cast<unsigned long long>(radius(lm + dl));
                    const unsigned long long rhs = sStrongS[k] * static_cast<unsigned long long>(radius(lm));
                    const bool earlier = dl < 0 || (dl == 0 && (dy < 0 || (dy == 0 && dx < 0)));
                    return earlier ? !(lhs > rhs) : !(lhs >= rhs);
                };
                if (ns > NS_HASH) {
                    // a long list (the mark of a ring-centre tile, the slowest work of a launch):
                    // the strong voxels go into an open-addressing table keyed by voxel, and each
                    // candidate looks up its 26 neighbours, one task per candidate and level
                    // offset.  The table takes the hotspot list's storage, which this window does
                    // not read again; when windows relist from the hotspot list, it takes the
                    // histogram's, which is not read again in this chunk.
                    uint32_t* const sTab = in_hist ? sA : reinterpret_cast<uint32_t*>(sScratch);
                    for (int i = tid; i < HT; i += NT) sTab[i] = 0xffffffffu;
                    __syncthreads();
                    for (int j = tid; j < ns; j += NT) {
                        const uint32_t e = sStrongId[j];
                        const uint32_t key = ((e >> 16) << KEY_BITS) | (e & 0xffffu);     // distinct per voxel
                        // at most SCAP of HT slots are taken, so the probe ends
                        for (uint32_t slot = strong_slot(key);; slot = (slot + 1) & (HT - 1))
                            if (atomicCAS(&sTab[slot], 0xffffffffu, (key << 16) | static_cast<uint32_t>(j)) == 0xffffffffu)
                                break;
                    }
                    __syncthreads();
                    for (int task = tid; task < 3 * ns; task += NT) {
                        const int j = task / 3, dl = task - 3 * j - 1;
                        int li, lm, sxr, syr;
                        if (!candidate(j, li, lm, sxr, syr)) continue;
                        const int nl = li + dl;
                        if (nl < 0 || nl >= nlev) continue;
                        const unsigned long long sv = sStrongS[j];
                        bool peak = true;
#pragma unroll
                        for (int o = 0; o < 9; ++o) {
                            const int dy = o / 3 - 1, dx = o % 3 - 1;
                            if (dl == 0 && dy == 0 && dx == 0) continue;
                            // 1 <= sxr, syr <= T: the neighbour lies in the score region's index range
                            const uint32_t key = (static_cast<uint32_t>(nl) << KEY_BITS) |
                                                 static_cast<uint32_t>((syr + dy) * SR + sxr + dx);
                            for (uint32_t slot = strong_slot(key);; slot = (slot + 1) & (HT - 1)) {
                                const uint32_t v = sTab[slot];
                                if (v == 0xffffffffu) break;                      // not strong
                                if ((v >> 16) == key) {
                                    if (beats(sv, lm, static_cast<int>(v & 0xffffu), dl, dy, dx)) peak = false;
                                    break;
                                }
                            }
                        }
                        if (!peak) sBad[j] = 1;
                    }
                    __syncthreads();
                    for (int j = tid; j < ns; j += NT) {
                        int li, lm, sxr, syr;
                        if (candidate(j, li, lm, sxr, syr) && !sBad[j]) emit(j, lm, sxr, syr);
                    }
                } else {
                    // a short list: G lanes per strong voxel, each comparing a slice of about two
                    // entries of the list (one lane when the list holds at most four)
                    const int gs = ns <= 4 ? 0 : min(4, 31 - __builtin_clz(static_cast<unsigned>(ns - 1)));
                    const int G = 1 << gs;
                    for (int task = tid; task < (ns << gs); task += NT) {
                        const int j = task >> gs, g = task & (G - 1);
                        int li, lm, sxr, syr;
                        if (!candidate(j, li, lm, sxr, syr)) continue;
                        // the neighbours that matter are strong too (a weaker one cannot win), so
                        // the comparison runs over the window's strong list
                        const unsigned long long sv = sStrongS[j];
                        bool peak = true;
                        for (int k = g; k < ns && peak; k += G) {
                            if (k == j) continue;
                            const uint32_t eu = sStrongId[k];
                            const int dl = static_cast<int>(eu >> 16) - li;
                            const int su_idx = static_cast<int>(eu & 0xffffu);
                            const int dy = su_idx / SR - syr, dx = su_idx % SR - sxr;
                            if (dl < -1 || dl > 1 || dy < -1 || dy > 1 || dx < -1 || dx > 1) continue;
                            if (beats(sv, lm, k, dl, dy, dx)) peak = false;
                        }
                        if (G == 1) {
                            if (peak) emit(j, lm, sxr, syr);
                        } else if (!peak) {
                            sBad[j] = 1;
                        }
                    }
                    if (G > 1) {
                        __syncthreads();
                        for (int j = tid; j < ns; j += NT) {
                            int li, lm, sxr, syr;
                            if (candidate(j, li, lm, sxr, syr) && !sBad[j]) emit(j, lm, sxr, syr);
                        }
                    }
                }
                wlo = whi;
            }
            if (windows && !per_level) __syncthreads();       // the table in the histogram is done
            if (PHASES) {                                     // the profiling instance splits here
                __syncthreads();
                stamp(PH_PEAK);
            }
            const bool last = rc1 > L - 2;
            if (!last) {
                rc0 = rc1;
                rc1 = chunk_end(rc0, carry ? 2 : 0);
                prepare(rc0, rc1, carry ? 2 : 0);
            }
            __syncthreads();
            stamp(PH_PREP);
            if (last) break;
        }
    }
    if (PHASES && tid == 0) {
        // per workgroup: each phase's clocks, its lifetime, its tiles; the longest and the
        // shortest lifetime over the workgroups
        const unsigned long long life = __builtin_readcyclecounter() - ph_start;
        for (int i = 0; i < PH_COUNT; ++i) atomicAdd(&a.phase_clocks[i], ph_acc[i]);
        atomicAdd(&a.phase_clocks[PH_COUNT], life);
        atomicAdd(&a.phase_clocks[PH_COUNT + 1], static_cast<unsigned long long>(ph_tiles));
        atomicMax(&a.phase_clocks[PH_COUNT + 2], life);
        atomicMin(&a.phase_clocks[PH_COUNT + 3], life);
    }
    if (a.stats) {
        unsigned long long v = st_votes, tp = st_taps;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            v += __shfl_xor(v, o, 64);
            tp += __shfl_xor(tp, o, 64);
        }
        // per wave, then per block: one device atomic per counter and block (thousands of
        // same-address atomics at the end of the launch would serialise behind the last tile)
        __shared__ unsigned long long sRed[NW][2];
        if (lane == 0) {
            sRed[tid >> 6][0] = v;
            sRed[tid >> 6][1] = tp;
        }
        __syncthreads();
        if (tid == 0) {
            for (int w = 1; w < NW; ++w) {
                v += sRed[w][0];
                tp += sRed[w][1];
            }
            atomicAdd(&a.stats[0], v);
            atomicAdd(&a.stats[3], tp);
            atomicAdd(&a.stats[1], st_hot);
            atomicAdd(&a.stats[2], st_strong);
        }
    }
}

// ---- tile order ------------------------------------------------------------------------

constexpr int CNT_ = 256;         // threads of the cost kernel
constexpr int CWIN = 2048;        // tiles of a workgroup's window (counted in LDS)
constexpr int ONT = 1024;         // threads of the order kernel
constexpr int NCLASS = 128;       // cost classes (4 per octave)

// One workgroup per chunk of COST_CHUNK bins; one task per (ridge, sign).  The sampled votes
// (levels COST_STEP / 2, 3 COST_STEP / 2, ...) land within the last level's radius (plus
// rounding) of the chunk's strip, so they are counted in LDS over that window of tiles and
// added to the tiles' counters with one global atomic per (workgroup, tile).
__global__ __launch_bounds__(CNT_) void k_tile_cost(TileCostArgs a) {
    __shared__ uint32_t sPre[COST_CHUNK + 1];
    __shared__ uint32_t sCnt[CWIN];
    const int tid = threadIdx.x, lane = tid & 63;
    const int cg = static_cast<int>(blockIdx.x);
    int f = 0;
    for (int hi = a.nframes; hi - f > 1;) {
        const int mid = (f + hi) >> 1;
        if (a.frames[mid].chunk0 <= cg) f = mid; else hi = mid;
    }
    const FrameDesc fd = a.frames[f];
    const int64_t nbins = static_cast<int64_t>(fd.nbx) * fd.nby;
    const int64_t b0 = static_cast<int64_t>(cg - fd.chunk0) * COST_CHUNK;
    const int64_t blast = min(b0 + COST_CHUNK, nbins) - 1;
    if (tid < 64) {                      // ridges per bin of the chunk, as a prefix sum
        const uint32_t c = (tid < COST_CHUNK && b0 + tid < nbins)
                               ? min(a.bin_count[fd.bin0 + b0 + tid], static_cast<uint32_t>(BIN_CAP)) : 0u;
        const uint32_t inc = wave_incl_scan(c, lane);
        if (tid < COST_CHUNK) sPre[tid + 1] = inc;
        if (tid == 0) sPre[0] = 0u;
    }
    const int T = a.tile, W = fd.W, H = fd.H;
    const int tiles_x = (W + T - 1) / T;
    const int by0 = static_cast<int>(b0 / fd.nbx), by1 = static_cast<int>(blast / fd.nbx);
    const int bx0 = by0 == by1 ? static_cast<int>(b0 % fd.nbx) : 0;
    const int bx1 = by0 == by1 ? static_cast<int>(blast % fd.nbx) : fd.nbx - 1;
    const int reach = a.rbase + a.rstep * (a.nlevels - 1) + 2;
    const int wx0 = max(0, bx0 * BIN - reach) / T, wx1 = min(W - 1, bx1 * BIN + BIN - 1 + reach) / T;
    const int wy0 = max(0, by0 * BIN - reach) / T, wy1 = min(H - 1, by1 * BIN + BIN - 1 + reach) / T;
    const int nwx = wx1 - wx0 + 1;
    const bool in_lds = nwx * (wy1 - wy0 + 1) <= CWIN;
    for (int i = tid; i < CWIN; i += CNT_) sCnt[i] = 0u;
    __syncthreads();
    const uint32_t total = sPre[COST_CHUNK];
    const uint32_t mT = 0xffffffffu / static_cast<uint32_t>(T) + 1u;   // floor(v / T) = mulhi(v, mT), v < 2^16
    for (uint32_t task = tid; task < 2 * total; task += CNT_) {
        const uint32_t k = task >> 1;
        const int sg = static_cast<int>(task & 1u);
        int bi = 0;
        while (bi + 1 < COST_CHUNK && sPre[bi + 1] <= k) ++bi;
        const int64_t slot = (fd.bin0 + b0 + bi) * BIN_CAP + (k - sPre[bi]);
        const uint32_t xy = a.rxy[slot], q = a.rq[slot];
        const int x = xy & 0xffffu, y = xy >> 16;
        const int qx = static_cast<int16_t>(q & 0xffffu), qy = static_cast<int16_t>(q >> 16);
        const int sqx = sg ? -qx : qx, sqy = sg ? -qy : qy, rnd = sg ? 8191 : 8192;
        for (int l = COST_STEP / 2; l < a.nlevels; l += COST_STEP) {
            const int r = a.rbase + a.rstep * l;
            const int vx = x + ((r * sqx + rnd) >> 14), vy = y + ((r * sqy + rnd) >> 14);
            if (vx < 0 || vx >= W || vy < 0 || vy >= H) continue;
            const int tx = static_cast<int>(div_mulhi(static_cast<uint32_t>(vx), T, mT));
            const int ty = static_cast<int>(div_mulhi(static_cast<uint32_t>(vy), T, mT));
            if (in_lds && tx >= wx0 && tx <= wx1 && ty >= wy0 && ty <= wy1)
                atomicAdd(&sCnt[(ty - wy0) * nwx + (tx - wx0)], 1u);
            else
                atomicAdd(&a.cost[fd.vtile0 + ty * tiles_x + tx], 1u);
        }
    }
    __syncthreads();
    if (in_lds)
        for (int i = tid; i < nwx * (wy1 - wy0 + 1); i += CNT_)
            if (sCnt[i]) atomicAdd(&a.cost[fd.vtile0 + (wy0 + i / nwx) * tiles_x + wx0 + i % nwx], sCnt[i]);
}

// One workgroup: each counter read once (and cleared for the next launch), then the order, a
// counting sort over 4 classes per octave of the cost with the costliest class first (the
// order within a class is arbitrary: no result depends on the order).
__global__ __launch_bounds__(ONT) void k_tile_order(TileCostArgs a) {
    __shared__ uint8_t sCls[ORDER_MAX];
    __shared__ uint32_t sB[NCLASS];
    const int tid = threadIdx.x, lane = tid & 63, n = a.total_vtiles;
    for (int i = tid; i < NCLASS; i += ONT) sB[i] = 0u;
    __syncthreads();
    for (int t = tid; t < n; t += ONT) {
        const uint32_t c = a.cost[t];
        const int k = c == 0u ? 0 : min(NCLASS - 1, 1 + static_cast<int>(4.0f * __log2f(static_cast<float>(c))));
        sCls[t] = static_cast<uint8_t>(k);
        atomicAdd(&sB[k], 1u);
        a.cost[t] = 0u;
    }
    __syncthreads();
    if (tid < 64) {                                  // class starts, the costliest class first
        const uint32_t hiC = sB[NCLASS - 1 - 2 * tid], loC = sB[NCLASS - 2 - 2 * tid];
        const uint32_t inc = wave_incl_scan(hiC + loC, lane);
        sB[NCLASS - 1 - 2 * tid] = inc - hiC - loC;
        sB[NCLASS - 2 - 2 * tid] = inc - loC;
    }
    __syncthreads();
    for (int t = tid; t < n; t += ONT) a.order[atomicAdd(&sB[sCls[t]], 1u)] = static_cast<uint32_t>(t);
}

// Scatter a caller-given ridge list into the per-bin slots, checking what keeps the votes
// exact: pixels inside the frame, each listed once (one bit per pixel of its bin, taken by an
// atomic), with a direction code as step 1 makes them.  Any failure sets a flag and the host
// reports RD_E_INVALID.
__global__ __launch_bounds__(NT) void k_bin(BinArgs a) {
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * NT) {
        const int x = a.xy[2 * i], y = a.xy[2 * i + 1];
        const int qx = a.q[2 * i], qy = a.q[2 * i + 1];
        if (x < 0 || x >= a.W || y < 0 || y >= a.H) {
            atomicOr(a.flags, static_cast<uint32_t>(BIN_OFF_FRAME));
            continue;
        }
        if (!ridge_code_ok(qx, qy)) {
            atomicOr(a.flags, static_cast<uint32_t>(BIN_BAD_CODE));
            continue;
        }
        const int64_t bin = (int64_t)(y >> BIN_SHIFT) * a.nbx + (x >> BIN_SHIFT);
        const int lp = ((y & (BIN - 1)) << BIN_SHIFT) | (x & (BIN - 1));
        const uint32_t bit = 1u << (lp & 31);
        if (atomicOr(&a.pixel_mask[bin * 8 + (lp >> 5)], bit) & bit) {
            atomicOr(a.flags, static_cast<uint32_t>(BIN_DUPLICATE));
            continue;
        }
        const uint32_t pos = atomicAdd(&a.bin_count[bin], 1u);   // < BIN_CAP: distinct pixels of one bin
        if (pos >= static_cast<uint32_t>(BIN_CAP)) {
            atomicOr(a.flags, static_cast<uint32_t>(BIN_OVERFLOW));
            continue;
        }
        const int64_t slot = bin * BIN_CAP + pos;
        a.rxy[slot] = static_cast<uint32_t>(x) | (static_cast<uint32_t>(y) << 16);
        a.rq[slot] = (static_cast<uint32_t>(static_cast<uint16_t>(qx))) | (static_cast<uint32_t>(static_cast<uint16_t>(qy)) << 16);
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

hipError_t launch_tile_cost(const TileCostArgs& a, int total_chunks, hipStream_t s) {
    if (a.total_vtiles <= 0 || a.total_vtiles > ORDER_MAX || total_chunks <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_tile_cost, dim3(total_chunks), dim3(CNT_), 0, s, a);
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(ONT), 0, s, a);
    return hipGetLastError();
}

size_t vote_lds_bytes(int tile, int nlev_max, int kmax) {
    const int side = tile + 2 + 2 * kmax;
    const size_t plane = (size_t)((side + 8) & ~7) * side;
    return ((nlev_max * plane * 2 + 15) / 16) * 16;
}

hipError_t vote_prepare() {
    // every instance may take the whole opted-in dynamic LDS
    const void* fns[] = {reinterpret_cast<const void*>(&k_vote<VOTE_TILE_RIDGE, false>),
                         reinterpret_cast<const void*>(&k_vote<VOTE_TILE_RIDGE, false, true>),
                         reinterpret_cast<const void*>(&k_vote<VOTE_TILE_RIDGE, true>),
                         reinterpret_cast<const void*>(&k_vote<VOTE_TILE_EDGE, false>),
                         reinterpret_cast<const void*>(&k_vote<VOTE_TILE_EDGE, false, true>),
                         reinterpret_cast<const void*>(&k_vote<VOTE_TILE_EDGE, true>)};
    for (int i = 0; i < 6; ++i) {
        const int lds = vote_lds_max(i < 3 ? VOTE_TILE_RIDGE : VOTE_TILE_EDGE);
        const hipError_t e = hipFuncSetAttribute(fns[i], hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int T>
void launch_vote_t(const VoteArgs& a, size_t lds, bool dump, int blocks, hipStream_t s) {
    if (dump)
        hipLaunchKernelGGL((k_vote<T, true>), dim3(blocks), dim3(NT), lds, s, a);
    else if (a.phase_clocks)
        hipLaunchKernelGGL((k_vote<T, false, true>), dim3(blocks), dim3(NT), lds, s, a);
    else
        hipLaunchKernelGGL((k_vote<T, false>), dim3(blocks), dim3(NT), lds, s, a);
}

hipError_t launch_vote(const VoteArgs& a, size_t lds, bool dump, int blocks, hipStream_t s) {
    if (a.total_vtiles <= 0 || a.nlevels < 3) return hipSuccess;
    if (lds > static_cast<size_t>(vote_lds_max(a.tile))) return hipErrorInvalidValue;   // beyond the opted-in size
    if (lds < static_cast<size_t>(VOTE_TABLE_BYTES)) lds = VOTE_TABLE_BYTES;
    if (blocks > a.total_vtiles) blocks = a.total_vtiles;   // persistent blocks take tiles from the queue
    VoteArgs b = a;
    b.hist_bytes = static_cast<int32_t>(lds);                 // the kernel cuts its level chunks to fit
    if (a.tile == VOTE_TILE_RIDGE) launch_vote_t<VOTE_TILE_RIDGE>(b, lds, dump, blocks, s);
    else if (a.tile == VOTE_TILE_EDGE) launch_vote_t<VOTE_TILE_EDGE>(b, lds, dump, blocks, s);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

__global__ void k_zero(uint32_t* p, int n, uint32_t* p2, int n2) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n + n2; i += gridDim.x * blockDim.x) {
        if (i < n) p[i] = 0u;
        else p2[i - n] = 0u;
    }
}

// Zeroing by a kernel rather than a memset node keeps captured graphs replay-safe.
hipError_t launch_zero2(uint32_t* p, int n, uint32_t* p2, int n2, hipStream_t s) {
    if (n < 0 || n2 < 0 || n + n2 <= 0) return hipSuccess;
    const int blocks = (n + n2 + 255) / 256 < 64 ? (n + n2 + 255) / 256 : 64;
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, p, n, p2, n2);
    return hipGetLastError();
}

hipError_t launch_zero(uint32_t* p, int n, hipStream_t s) { return launch_zero2(p, n, nullptr, 0, s); }

hipError_t launch_bin(const BinArgs& a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    int64_t blocks = (a.n + NT - 1) / NT;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_bin, dim3(static_cast<unsigned>(blocks)), dim3(NT), 0, s, a);
    return hipGetLastError();
}

}  // namespace rd
