// Internal declarations shared by the HIP sources of the ridge-directed Hough library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ridge_detect.h"

namespace rd {

// Ridge pixels are stored per 16x16 pixel bin, in BIN_CAP slots per bin, so that the
// vote and fit kernels can gather the ridges near any region without a global sort.
constexpr int BIN = 16;
constexpr int BIN_SHIFT = 4;
constexpr int BIN_CAP = BIN * BIN;

// A caller-given ridge direction code must be what step 1 produces: rint(2^14 X_-) of a
// unit vector, so |q|^2 lies within 2 * 2^14 * (|cos| + |sin|) / 2 + 1/2 <= 23171 of 2^28
// (accepted: within 2^15), in canonical sign (qy > 0, or qy == 0 and qx > 0).  With such
// codes and distinct pixels a voxel at level r takes at most one vote per lattice offset
// that rho(r, q) can reach, which keeps the u16 vote counters and the 32-bit band sums of
// the score exact.
constexpr uint32_t Q_UNIT2 = 1u << 28;
constexpr uint32_t Q_UNIT2_TOL = 1u << 15;
__host__ __device__ inline bool ridge_code_ok(int qx, int qy) {
    const uint32_t n2 = static_cast<uint32_t>(qx * qx) + static_cast<uint32_t>(qy * qy);   // <= 2^31
    const uint32_t dev = n2 > Q_UNIT2 ? n2 - Q_UNIT2 : Q_UNIT2 - n2;
    return dev <= Q_UNIT2_TOL && (qy > 0 || (qy == 0 && qx > 0));
}

constexpr int RG_MAX = 16;   // Gaussian radius ceil(4 sigma) limit (sigma <= 4)
constexpr int K_MAX = 24;    // smoothing window half-width limit
constexpr int R_LIMIT = 126; // largest level radius R_LIMIT + 1: keeps u16 vote counts and u64 scores exact
constexpr int R_STEP_MAX = 16;

// The radius step of a parameter set (0 reads as 1).
inline int param_rstep(const rd_params& p) { return p.r_step < 1 ? 1 : p.r_step; }
constexpr int MAX_DIM = 65535;

// One frame of a launch: where its pixels are and where its tiles / bins start in the
// launch-wide numbering.  A plain detection is a launch with one frame.
struct FrameDesc {
    const void* img;
    int64_t pitch;       // bytes
    int32_t W, H;
    int32_t tile0;       // first stencil tile of this frame
    int32_t vtile0;      // first vote tile of this frame
    int64_t bin0;        // first ridge bin of this frame
    int32_t nbx, nby;    // bins per row / column
    int32_t peak0;       // first peak slot of this frame
    int32_t chunk0;      // first COST_CHUNK-bin chunk of this frame (the tile-cost pass's work units)
};

constexpr int FRAMES_LDS = 64;   // frame tables up to this size are read into LDS by the kernels

struct Peak {
    int32_t a, b, r, frame;
    uint64_t s;          // integer smoothed score S_int
};

struct StencilArgs {
    const FrameDesc* frames;
    int32_t nframes;
    int32_t total_tiles;
    double g[RG_MAX + 1];    // g[0] centre tap, g[i] = g[-i]; zero beyond the radius
    double k_threshold;
    int32_t edge;            // 1: directed edges (m = -|grad I|, unit-gradient codes); 0: ridges
    int32_t fp32;            // 1: float32 filters on the tile-mean-offset image; 0: float64
    uint32_t* rxy;           // ridge (x | y << 16) per slot
    uint32_t* rq;            // ridge (qx & 0xffff | qy << 16) per slot
    float* rk;               // ridge k_- per slot
    uint32_t* bin_count;     // ridges per bin
    float* k_dense;          // dense outputs (stage mode, single frame)
    int16_t* q_dense;
    double* hess_dense;      // dense mode: Ixx, Iyy, Ixy planes [3][H][W] (may be null)
    unsigned long long* ridge_total;   // statistics: ridges found (may be null)
};

struct VoteArgs {
    const FrameDesc* frames;
    int32_t nframes;
    int32_t total_vtiles;
    int32_t hist_bytes;       // dynamic LDS of the launch: histogram planes of a level chunk (set by launch_vote)
    const uint32_t* rxy;
    const uint32_t* rq;
    const uint32_t* bin_count;
    int32_t lbase;            // radius of level 0: r_min - r_step
    int32_t r_step;           // level i has radius lbase + r_step i
    int32_t nlevels;          // L = (r_max - r_min) / r_step + 3
    int32_t vote_threshold;
    const uint32_t* wtab;        // [level][K_MAX + 1] 15-bit weight factors
    const int32_t* ktab;         // [level] window half-width
    const uint64_t* thr;         // [level] integer score threshold
    Peak* peaks;
    uint32_t* peak_count;        // per frame
    int32_t max_peaks;           // per frame
    uint32_t* error;             // bit 0: a work item had more strong voxels than it holds
    uint32_t* tile_counter;      // work queue of vote tiles (zero before the launch)
    unsigned long long* stats;   // [votes, hotspots, strong] accumulated (may be null)
    uint32_t* acc_dump;          // stage mode (single frame): dense [L][H][W]
    uint64_t* score_dump;
    const uint32_t* tile_order;  // [total_vtiles] the queue's tiles, estimated costliest first (may be null)
    unsigned long long* phase_clocks;  // profiling instance: [PH_COUNT + 4] (null: the plain kernel)
    unsigned long long* tile_clocks;   // profiling instance, may be null: per tile [workgroup,
                                       // queue position, clock at start, clock at end]
    int32_t tile;                // T of the T x T vote tiles (VOTE_TILE_RIDGE or VOTE_TILE_EDGE)
};

// Phases of the vote kernel's profiling instance (clocks summed over workgroups), then the
// workgroups' summed lifetime, the tiles, the longest and the shortest lifetime
enum { PH_SETUP = 0, PH_STAGE, PH_SORT, PH_VOTE, PH_SCORE, PH_STRONG, PH_PEAK, PH_PREP, PH_COUNT };

// The tile-cost pass: every (ridge, sign) casts its vote at one level in COST_STEP into a
// per-tile counter (the tile that holds the vote), an estimate of the tiles' vote work; a
// second kernel orders the tiles by decreasing cost class.  Launches with more
// than ORDER_MAX vote tiles are not ordered (with many tiles per workgroup the queue's tail is
// short anyway).
constexpr int COST_CHUNK = 8;     // bins per workgroup of the counting kernel
constexpr int COST_STEP = 8;      // levels per sampled vote
constexpr int ORDER_MAX = 8192;   // vote tiles of an ordered launch
struct TileCostArgs {
    const FrameDesc* frames;
    int32_t nframes;
    const uint32_t* rxy;
    const uint32_t* rq;
    const uint32_t* bin_count;
    int32_t rbase, rstep, nlevels;
    int32_t total_vtiles;        // <= ORDER_MAX
    int32_t tile;                // T of the vote tiles
    uint32_t* cost;              // [ORDER_MAX]: the tiles' counters, zero before the counting kernel and
                                 // cleared again by the order kernel
    uint32_t* order;             // [total_vtiles]
};
hipError_t launch_tile_cost(const TileCostArgs& a, int total_chunks, hipStream_t s);

struct FitArgs {
    const FrameDesc* frames;
    uint32_t* counts_out;        // per frame ring count, then the vote error flag (host mapped)
    const uint32_t* error;
    const uint32_t* rxy;
    const uint32_t* bin_count;
    const Peak* peaks;
    const uint32_t* peak_count;  // per frame
    int32_t nframes;
    int32_t max_peaks;
    int32_t w;
    int32_t min_pts;
    rd_ring* rings;              // [nframes * max_peaks], slot = frame peak0 + rank
    const unsigned long long* stats_in;   // statistics counters, copied by block 0 (may be null)
    unsigned long long* stats_out;        // (host mapped)
    int32_t nstats;
};

// ---- encoded ridge streams (the compact transfer form of a frame's ridges)
constexpr int RIDGE_CHUNK = 256;          // bins per work unit of the encode / decode kernels
constexpr uint32_t RIDGE_MAGIC = 0x31524452u;   // "RDR1"
// byte size of one frame's stream: header, u16 per bin, u8 per ridge, pad to 4, u32 per ridge,
// pad to 16
__host__ __device__ inline int64_t ridge_stream_bytes(int64_t n, int64_t nbins) {
    const int64_t qoff = (16 + 2 * nbins + n + 3) & ~static_cast<int64_t>(3);
    return (qoff + 4 * n + 15) & ~static_cast<int64_t>(15);
}
__host__ __device__ inline int64_t ridge_stream_qoff(int64_t n, int64_t nbins) {
    return (16 + 2 * nbins + n + 3) & ~static_cast<int64_t>(3);
}

struct RidgeCodeArgs {
    const FrameDesc* frames;
    int32_t nframes;
    const uint32_t* chunk0;      // [nframes + 1] first chunk of each frame (launch-wide numbering)
    uint32_t* cbase;             // [chunks] record index of each chunk's first ridge in its frame
    uint32_t* frame_n;           // [nframes] ridges per frame
    uint32_t* flags;             // decode: bit 0 malformed stream (counts, size), bit 1 off-frame
                                 // pixel, bit 2 bad direction code, bit 3 repeated pixel
    uint32_t* rxy;               // the context's ridge bins
    uint32_t* rq;
    float* rk;
    uint32_t* bin_count;
    uint8_t* enc;                // encode: output buffer; decode: staged streams
    int64_t capacity;            // encode: bytes of enc
    int64_t* offsets;            // [nframes + 1] stream byte offsets (encode: written; decode: read)
};

hipError_t launch_ridge_encode(const RidgeCodeArgs& a, int total_chunks, hipStream_t s);
hipError_t launch_ridge_decode(const RidgeCodeArgs& a, int total_chunks, hipStream_t s);

// flags of a caller-given ridge list (BinArgs::flags)
enum { BIN_OVERFLOW = 1, BIN_OFF_FRAME = 2, BIN_BAD_CODE = 4, BIN_DUPLICATE = 8 };

struct BinArgs {
    const int32_t* xy;
    const int16_t* q;
    int64_t n;
    int32_t W, H, nbx;
    uint32_t* rxy;
    uint32_t* rq;
    float* rk;
    uint32_t* bin_count;
    uint32_t* pixel_mask;   // 8 words (one bit per pixel) per 16 x 16 bin, zero before the launch
    uint32_t* flags;
};

// Launchers (return hipSuccess or the launch error).
// stencil tile shapes: variant 0 = 64 x 32 (64 x 16 for Gaussian radius > 8), 1 = 32 x 32,
// 2 = 64 x 16; the dense stage output always uses variant 0
constexpr int STENCIL_VARIANTS = 3;
void stencil_tile_dims(int variant, int rg, bool dense, int* tw, int* th);
hipError_t launch_stencil(const StencilArgs& a, int dtype, int rg, int variant, bool dense, hipStream_t s);

// Vote tiles of T x T pixels: 40 for directed ridges; 32 for directed edges, whose frames
// list about twice the hotspots per area, so that a tile's list overflows into the
// level-by-level fallback less often.  The tile size changes the work's split, no result.
constexpr int VOTE_TILE_RIDGE = 40, VOTE_TILE_EDGE = 32;
inline int vote_tile_for(int32_t measure) { return measure == RD_MEASURE_EDGE ? VOTE_TILE_EDGE : VOTE_TILE_RIDGE; }
constexpr int VOTE_LDS_MAX = RD_VOTE_LDS_KB_MAX * 1024;   // dynamic LDS of the vote kernel, the largest instance
// what each instance's static LDS (about 70 KB, and 6.5 KB more hotspot list for the larger
// tile) leaves of a compute unit's 160 KiB; a tuning budget above it is clamped
inline int vote_lds_max(int tile) { return tile == VOTE_TILE_EDGE ? VOTE_LDS_MAX : 83 * 1024; }
constexpr int VOTE_NLEV_MAX = 20;          // accumulator levels per level chunk
constexpr int VOTE_TABLE_BYTES = 8192;     // least dynamic LDS of a vote launch (the peak test's table)
size_t vote_lds_bytes(int tile, int nlev_max, int kmax);
hipError_t vote_prepare();   // one-time kernel attributes (outside any graph capture)
hipError_t launch_vote(const VoteArgs& a, size_t lds, bool dump, int blocks, hipStream_t s);
hipError_t launch_zero(uint32_t* p, int n, hipStream_t s);
hipError_t launch_zero2(uint32_t* p, int n, uint32_t* p2, int n2, hipStream_t s);   // both ranges, one launch
constexpr int FIT_GRID = 512;   // workgroups of the fit kernel (each takes peaks in turn)
hipError_t launch_fit(const FitArgs& a, int blocks, hipStream_t s);
hipError_t launch_bin(const BinArgs& a, hipStream_t s);
hipError_t launch_gather(const uint32_t* rxy, const uint32_t* rq, const float* rk, const uint32_t* bin_count,
                         const int64_t* offsets, int64_t nbins, int32_t* xy, int16_t* q, float* k, hipStream_t s);

// ---- differentiable path (soft accumulator, adjoints, ring-profile fit)

constexpr int SOFT_TILE = 32;     // accumulator tile side owned by one workgroup
constexpr int SOFT_LEVELS = 8;    // accumulator levels per workgroup (32 KB of LDS)

// Ridges of a soft launch binned by 16x16 pixel bins, with their splat geometry.
struct SoftBinArgs {
    const int32_t* xy;       // [n][2] ridge pixels
    const double* hess;      // [n][3] Ixx, Iyy, Ixy at the ridge pixels
    int64_t n;
    int32_t W, H, nbx;
    uint32_t* sxy;           // per slot: x | y << 16
    double* sux;             // per slot: X_- (continuous)
    double* suy;
    float* sw;               // per slot: w = -k_-
    uint32_t* bin_count;
    uint32_t* flags;         // bit 0: a bin overflowed, bit 1: a ridge off the frame
};

struct SoftFwdArgs {
    const uint32_t* sxy;
    const double* sux;
    const double* suy;
    const float* sw;
    const uint32_t* bin_count;
    int32_t W, H, nbx, nby;
    int32_t r_lo, L;         // levels r_lo .. r_lo + L - 1
    float* acc;              // [L][H][W]
};

struct SoftBwdArgs {
    const int32_t* xy;
    const double* hess;
    int64_t n;
    int32_t W, H, r_lo, L;
    const float* grad_acc;   // [L][H][W]
    double* grad_hess;       // [n][3]
    uint32_t* n_iso;         // near-isotropic ridges whose X_- term was dropped
};

// One pass of a transposed 1D correlation with reflect-101 fold-back along x (dir 0) or
// y (dir 1).  sum = 0: out[c] = scale T_c(in[c]) for each component; sum = 1:
// out[0] = scale sum_c T_c(in[c]); accumulate adds into out instead of overwriting.
constexpr int ADJ_TAPS = 2 * RG_MAX + 1;
struct AdjPassArgs {
    const float* in[3];
    float* out[3];
    double taps[3][ADJ_TAPS];
    int32_t ncomp, R, W, H, sum, accumulate;
    double scale;
};

struct ScatterArgs {
    const int32_t* xy;
    const double* grad_hess;
    int64_t n;
    int32_t W, H;
    float* planes;           // [3][H][W], zeroed before
};

// A frame of a ring-profile launch.
struct RingFrame {
    const void* img;
    int64_t pitch;           // bytes
    int32_t W, H, dtype, pad;
    int64_t grad_off;        // backward: first element of this frame's [H][W] plane in grad_img
};

constexpr int RING_FRAMES_MAX = 64;   // frames of one ring-profile launch (kernel arguments)
struct RingArgs {
    RingFrame frames[RING_FRAMES_MAX];
    int32_t nframes;
    const int32_t* frame_of; // [m] frame of each ring (null: frame 0); rings of other indices are skipped
    int64_t m;
    const double* theta;     // [m][3] cx, cy, r
    const double* theta0;    // [m][3] ring that fixes the window
    double s, halfwidth;     // profile sigma, window half-width 3 s + 2
    double* loss;            // [m]
    double* ab;              // [m][2] A, B (may be null)
    const double* grad_loss; // backward: [m] upstream gradient
    float* grad_img;         // backward: the frames' [H][W] planes from RingFrame.grad_off, added into (may be null)
    double* grad_theta;      // backward: [m][3]
    int32_t iters;           // refinement steps, at most
    double tol;              // a step whose update is within tol in every component is the last
    double lam0, lam_down, lam_up;
    double* theta_out;       // refinement result [m][3]
    int32_t* steps_out;      // steps taken [m] (may be null)
};

hipError_t launch_hess_gather(const double* planes, int W, int H, const int32_t* xy, int64_t n, double* hess,
                              hipStream_t s);
hipError_t launch_soft_bin(const SoftBinArgs& a, hipStream_t s);
hipError_t launch_soft_forward(const SoftFwdArgs& a, hipStream_t s);
hipError_t launch_soft_backward(const SoftBwdArgs& a, hipStream_t s);
hipError_t launch_scatter_grad_hess(const ScatterArgs& a, hipStream_t s);
hipError_t launch_adj_pass(const AdjPassArgs& a, int dir, hipStream_t s);
hipError_t launch_fill_f32(float* p, int64_t n, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, hipStream_t s);
hipError_t launch_fit_loss(const RingArgs& a, bool backward, hipStream_t s);
hipError_t launch_refine(const RingArgs& a, hipStream_t s);

}  // namespace rd
