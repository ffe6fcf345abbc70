// Host-side context of the ridge-directed Hough library, shared by the host sources: the
// status macros, the cached per-level tables, the key of a captured launch sequence and the
// context that owns every device buffer.
#pragma once

#include <cstring>
#include <vector>

#include "rd_internal.h"

#define RD_HIP(call)                                   \
    do {                                               \
        if ((call) != hipSuccess) return RD_E_DEVICE;  \
    } while (0)

#define RD_TRY(call)                      \
    do {                                  \
        const rd_status st_ = (call);     \
        if (st_ != RD_OK) return st_;     \
    } while (0)

namespace rd {

// Level tables: level i has radius lbase + rstep i, i = 0 .. L - 1 (radii r_min - s .. past
// r_max by one step); the chunk boundaries are level indices.
struct LevelTables {
    int lbase = 0, rstep = 1, L = 0;
    std::vector<uint32_t> wtab;      // L x (K_MAX + 1)
    std::vector<int32_t> ktab;       // L
    std::vector<uint64_t> thr;       // L
    size_t lds = 0;                  // vote-histogram storage (dynamic LDS) of the launch
};

// The same tables in fixed-size arrays (no heap), for the entry point that allocates nothing.
struct FixedTables {
    int lbase = 0, rstep = 1, L = 0;
    uint32_t wtab[(R_LIMIT + 3) * (K_MAX + 1)];
    int32_t ktab[R_LIMIT + 3];
    uint64_t thr[R_LIMIT + 3];
    size_t lds = 0;
};

// Level tables of *p for a vote-histogram LDS budget of `budget` bytes.
void build_fixed_tables(const rd_params& p, FixedTables& t, size_t budget);

// Ridge-kernel arguments that depend on the parameters only (smoothing taps, threshold,
// measure); the caller fills in the output pointers.
StencilArgs stencil_args_for(const rd_params& p, const FrameDesc* frames, int nframes, int total_tiles);

inline bool same_params(const rd_params& a, const rd_params& b) {
    return std::memcmp(&a, &b, sizeof(rd_params)) == 0;
}

// Everything a captured launch sequence bakes into its kernel arguments and grids; frame
// pointers and sizes live in the device-side descriptor table and may change freely.
struct GraphKey {
    int nframes = 0, dtype = 0, rg = 0, variant = 0, total_tiles = 0, total_vtiles = 0, blocks = 0;
    int bin_chunks = 0;
    bool timing = false;   // the graph holds the timing events' record nodes
    size_t lds = 0;
    rd_params params{};
    bool operator==(const GraphKey& o) const {
        return nframes == o.nframes && dtype == o.dtype && rg == o.rg && variant == o.variant && timing == o.timing &&
               total_tiles == o.total_tiles && total_vtiles == o.total_vtiles &&
               blocks == o.blocks && lds == o.lds && bin_chunks == o.bin_chunks && same_params(params, o.params);
    }
};

struct SoftState;                     // scratch of the differentiable path, made on first use
void soft_state_free(SoftState* s);

}  // namespace rd

struct rd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int cus = 0;
    int max_w = 0, max_h = 0, max_peaks = 0, max_frames = 0;
    int64_t max_batch_px = 0;
    int64_t max_bins = 0;
    // device scratch
    void* d_stage = nullptr;            // host frames are staged here (4 bytes per pixel)
    uint32_t* d_rxy = nullptr;          // ridge records, BIN_CAP slots per 16x16 bin
    uint32_t* d_rq = nullptr;
    float* d_rk = nullptr;
    uint32_t* d_bin_count = nullptr;
    rd::Peak* d_peaks = nullptr;        // max_peaks per frame
    uint32_t* d_counts = nullptr;       // [0, mf) peaks per frame, [mf] bin overflow, [mf+1] vote error,
                                        // [mf+2] vote tile queue
    unsigned long long* d_stats = nullptr;
    rd::FrameDesc* d_frames = nullptr;
    uint32_t* d_wtab = nullptr;
    int32_t* d_ktab = nullptr;
    uint64_t* d_thr = nullptr;
    int64_t* d_offsets = nullptr;       // stage gather offsets (per bin of one frame)
    uint32_t* d_pixmask = nullptr;      // caller ridge lists: one bit per pixel of one frame's bins
    // encoded ridge streams: per-chunk record bases (256 bins a chunk), per-frame ridge counts,
    // first chunk of each frame and an error flag (d_cmeta), stream byte offsets (d_eoff)
    uint32_t* d_cbase = nullptr;
    uint32_t* d_cmeta = nullptr;
    int64_t* d_eoff = nullptr;
    int64_t max_chunks = 0;
    // tile order of the vote kernel (launches of up to ORDER_MAX vote tiles): per-tile cost
    // estimates (zero between launches) and the order
    uint32_t* d_tcost = nullptr;
    unsigned long long* d_phase = nullptr;   // rd_profile_vote_phases: the clocks (allocated on first use)
    bool phase_on = false;
    unsigned long long* d_trec = nullptr;     // rd_profile_vote_tiles: 4 words per vote tile
    int64_t trec_cap = 0;                     // tiles d_trec holds
    bool trec_on = false;
    int vtile = rd::VOTE_TILE_RIDGE;        // vote tile of the parameters the tables were set up for
    uint32_t* d_torder = nullptr;
    int n_chunks = 0;                   // COST_CHUNK-bin chunks of the current launch's frames
    // pinned host memory; rings and counts are written by the fit kernel through mappings
    rd_ring* h_rings = nullptr;
    rd_ring* dh_rings = nullptr;
    uint32_t* h_counts = nullptr;
    uint32_t* dh_counts = nullptr;
    rd::FrameDesc* h_frames = nullptr;
    uint64_t* h_stats = nullptr;        // written by the fit kernel through dh_stats
    uint64_t* dh_stats = nullptr;
    // the descriptors d_frames holds (frames_dev_n of them, 0: unknown): an unchanged set is
    // not uploaded again
    std::vector<rd::FrameDesc> frames_dev;
    int frames_dev_n = 0;
    // kernel timing
    bool timing = false;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    double t_ms[3] = {0, 0, 0};
    int64_t t_n[3] = {0, 0, 0};
    uint64_t t_calls = 0;   // detection calls with timing on since the last reset (every eighth is timed)
    // tuning and the cached level tables
    rd_tuning tune{0, RD_VOTE_LDS_KB_MAX, 1};
    rd_params tab_params{};
    size_t tab_budget = 0;
    bool tab_valid = false;
    rd::LevelTables tabs;
    // captured launch sequence
    hipGraphExec_t gexec[2] = {nullptr, nullptr};   // [1]: the graph with the timing events
    rd::GraphKey gkey[2];
    bool mark_now = false;                          // this call records the timing events
    int64_t last_stats[6] = {0, 0, 0, 0, 0, 0};
    // differentiable path
    rd::SoftState* soft = nullptr;
};

namespace rd {

// Shared host helpers (defined with the plain entry points).
int gauss_radius(float sigma);
int vote_tiles(int W, int H, int T);
rd_status check_frame(const rd_ctx* h, const rd_frame* f);
rd_status setup_frames(rd_ctx* h, const rd_frame* frames, int n, int rg, int variant, bool dense, int* total_tiles,
                       int* total_vtiles);
int assign_chunks(rd_ctx* h, int n);     // chunk0 of h_frames[0 .. n); returns (and keeps) the total
StencilArgs stencil_args(rd_ctx* h, const rd_params& p, int nframes, int total_tiles);
rd_status find_ridges(rd_ctx* h, const rd_frame* frame, const rd_params& p);
rd_status gather_ridges(rd_ctx* h, int32_t* xy, int16_t* q, float* k, int64_t capacity, int64_t* n);

}  // namespace rd
