// Host runtime and C ABI of the ridge-directed Hough library: parameter validation, the
// per-level tables (window half-widths, fixed-point weights, score thresholds, level
// chunks), context-owned device scratch, frame-descriptor tables for batches, HIP-graph
// capture and replay of the launch sequence, tuning and the entry points.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "rd_host.h"

using namespace rd;

namespace {

constexpr double TWO_PI = 6.283185307179586;
constexpr double S_SCALE = 1073741824.0;   // 2^30
constexpr int NSTATS = 8 + 64;             // u64: votes, hotspots, strong, taps, -, -, -, -, 64 ridge stripes

double level_sigma(const rd_params& p, int r) {
    return static_cast<double>(p.sig_slope) * r + static_cast<double>(p.sig_icpt);
}

int level_radius(const rd_params& p, int r) { return static_cast<int>(std::ceil(3.0 * level_sigma(p, r))); }

void build_tables(const rd_params& p, LevelTables& t, size_t budget) {
    FixedTables f;
    build_fixed_tables(p, f, budget);
    t.lbase = f.lbase;
    t.rstep = f.rstep;
    t.L = f.L;
    t.wtab.assign(f.wtab, f.wtab + static_cast<size_t>(f.L) * (K_MAX + 1));
    t.ktab.assign(f.ktab, f.ktab + f.L);
    t.thr.assign(f.thr, f.thr + f.L);
    t.lds = f.lds;
}

}  // namespace

namespace rd {

void build_fixed_tables(const rd_params& p, FixedTables& t, size_t budget) {
    t.rstep = param_rstep(p);
    t.lbase = p.r_min - t.rstep;
    t.L = (p.r_max - p.r_min) / t.rstep + 3;
    std::memset(t.wtab, 0, sizeof(t.wtab));
    for (int i = 0; i < t.L; ++i) {
        const int l = t.lbase + t.rstep * i;
        const double sg = level_sigma(p, l);
        const int K = level_radius(p, l);
        t.ktab[i] = K;
        for (int d = 0; d <= K; ++d)
            t.wtab[static_cast<size_t>(i) * (K_MAX + 1) + d] =
                static_cast<uint32_t>(std::floor(32768.0 * std::exp(-(double)(d * d) / (2.0 * sg * sg)) + 0.5));
        t.thr[i] = static_cast<uint64_t>(
            std::floor(static_cast<double>(p.peak_fraction) * TWO_PI * static_cast<double>(l) * S_SCALE));
    }
    // the vote kernel's histogram storage: the budget, or the largest chunk of one peak level
    // (three planes at the top level's window, K growing with the level) if that is larger.
    // The kernel cuts each tile's level chunks to fit.
    t.lds = std::max(budget, vote_lds_bytes(vote_tile_for(p.measure), 3, t.ktab[t.L - 1]));
}

StencilArgs stencil_args_for(const rd_params& p, const FrameDesc* frames, int nframes, int total_tiles) {
    StencilArgs a{};
    a.frames = frames;
    a.nframes = nframes;
    a.total_tiles = total_tiles;
    const double sg = p.sigma_smooth;
    const int R = gauss_radius(p.sigma_smooth);
    double sum = 0.0;
    double g[RG_MAX + 1] = {0};
    for (int i = 0; i <= R; ++i) {
        g[i] = std::exp(-(double)(i * i) / (2.0 * sg * sg));
        sum += (i == 0 ? 1.0 : 2.0) * g[i];
    }
    for (int i = 0; i <= RG_MAX; ++i) a.g[i] = i <= R ? g[i] / sum : 0.0;
    a.k_threshold = p.k_threshold;
    a.edge = p.measure == RD_MEASURE_EDGE ? 1 : 0;
    a.fp32 = p.curvature_fp32 ? 1 : 0;
    return a;
}

int gauss_radius(float sigma) { return static_cast<int>(std::ceil(4.0 * static_cast<double>(sigma))); }

int vote_tiles(int W, int H, int T) { return ((W + T - 1) / T) * ((H + T - 1) / T); }

int assign_chunks(rd_ctx* h, int n) {
    int tot = 0;
    for (int i = 0; i < n; ++i) {
        h->h_frames[i].chunk0 = tot;
        tot += static_cast<int>((static_cast<int64_t>(h->h_frames[i].nbx) * h->h_frames[i].nby + COST_CHUNK - 1) /
                                COST_CHUNK);
    }
    h->n_chunks = tot;
    return tot;
}

rd_status check_frame(const rd_ctx* h, const rd_frame* f) {
    if (!f || !f->data) return RD_E_INVALID;
    if (f->dtype != RD_U16 && f->dtype != RD_F32) return RD_E_INVALID;
    if (f->width < 32 || f->height < 32) return RD_E_INVALID;
    const int64_t esz = f->dtype == RD_U16 ? 2 : 4;
    if (f->pitch_bytes < f->width * esz || f->pitch_bytes % esz != 0) return RD_E_INVALID;
    if (f->width > h->max_w || f->height > h->max_h) return RD_E_TOO_LARGE;
    return RD_OK;
}

// Frame descriptors of a launch; host frames are copied into the staging area.
rd_status setup_frames(rd_ctx* h, const rd_frame* frames, int n, int rg, int variant, bool dense, int* total_tiles,
                       int* total_vtiles) {
    int tw = 0, th = 0;
    stencil_tile_dims(variant, rg, dense, &tw, &th);
    int tt = 0, tv = 0;
    int64_t bins = 0, staged = 0;
    for (int i = 0; i < n; ++i) {
        const rd_frame& f = frames[i];
        const int64_t esz = f.dtype == RD_U16 ? 2 : 4;
        FrameDesc fd{};
        fd.W = f.width;
        fd.H = f.height;
        if (f.on_device) {
            fd.img = f.data;
            fd.pitch = f.pitch_bytes;
        } else {
            char* dst = static_cast<char*>(h->d_stage) + staged;
            RD_HIP(hipMemcpy2DAsync(dst, f.width * esz, f.data, f.pitch_bytes, f.width * esz, f.height,
                                    hipMemcpyHostToDevice, h->stream));
            fd.img = dst;
            fd.pitch = f.width * esz;
            staged += ((static_cast<int64_t>(f.width) * f.height * esz + 255) / 256) * 256;
        }
        fd.tile0 = tt;
        fd.vtile0 = tv;
        fd.bin0 = bins;
        fd.nbx = (f.width + BIN - 1) / BIN;
        fd.nby = (f.height + BIN - 1) / BIN;
        fd.peak0 = i * h->max_peaks;
        h->h_frames[i] = fd;
        tt += ((f.width + tw - 1) / tw) * ((f.height + th - 1) / th);
        tv += vote_tiles(f.width, f.height, h->vtile);
        bins += static_cast<int64_t>(fd.nbx) * fd.nby;
    }
    if (bins > h->max_bins) return RD_E_TOO_LARGE;
    assign_chunks(h, n);
    // a call on the same frame buffers (the usual loop) finds its descriptors already there
    if (h->frames_dev_n != n || std::memcmp(h->frames_dev.data(), h->h_frames, n * sizeof(FrameDesc)) != 0) {
        RD_HIP(hipMemcpyAsync(h->d_frames, h->h_frames, n * sizeof(FrameDesc), hipMemcpyHostToDevice, h->stream));
        h->frames_dev.assign(h->h_frames, h->h_frames + n);
        h->frames_dev_n = n;
    }
    *total_tiles = tt;
    *total_vtiles = tv;
    return RD_OK;
}

StencilArgs stencil_args(rd_ctx* h, const rd_params& p, int nframes, int total_tiles) {
    StencilArgs a = stencil_args_for(p, h->d_frames, nframes, total_tiles);
    a.rxy = h->d_rxy;
    a.rq = h->d_rq;
    a.rk = h->d_rk;
    a.bin_count = h->d_bin_count;
    a.ridge_total = h->d_stats + 8;
    return a;
}


// Steps 1-2 on one frame: the ridges land in the context's bins.
rd_status find_ridges(rd_ctx* h, const rd_frame* frame, const rd_params& p) {
    const int rg = gauss_radius(p.sigma_smooth);
    int tt = 0, tv = 0;
    RD_TRY(setup_frames(h, frame, 1, rg, h->tune.stencil_tile, false, &tt, &tv));
    StencilArgs sa = stencil_args(h, p, 1, tt);
    sa.ridge_total = nullptr;
    RD_HIP(launch_stencil(sa, frame->dtype, rg, h->tune.stencil_tile, false, h->stream));
    return RD_OK;
}

// The binned ridges of the last single-frame launch as a list in bin order: per-bin counts
// come back to the host, which forms the offsets, then one gather kernel copies.
rd_status gather_ridges(rd_ctx* h, int32_t* xy, int16_t* q, float* k, int64_t capacity, int64_t* n) {
    const FrameDesc& fd = h->h_frames[0];
    const int64_t nbins = static_cast<int64_t>(fd.nbx) * fd.nby;
    std::vector<uint32_t> cnt(nbins);
    RD_HIP(hipMemcpyAsync(cnt.data(), h->d_bin_count, nbins * 4, hipMemcpyDeviceToHost, h->stream));
    RD_HIP(hipStreamSynchronize(h->stream));
    std::vector<int64_t> off(nbins);
    int64_t tot = 0;
    for (int64_t b = 0; b < nbins; ++b) {
        off[b] = tot;
        tot += cnt[b];
    }
    *n = tot;
    if (tot > capacity) return RD_E_TRUNCATED;
    if (tot == 0) return RD_OK;
    if (!xy && !q && !k) return RD_OK;
    RD_HIP(hipMemcpyAsync(h->d_offsets, off.data(), nbins * sizeof(int64_t), hipMemcpyHostToDevice, h->stream));
    RD_HIP(launch_gather(h->d_rxy, h->d_rq, h->d_rk, h->d_bin_count, h->d_offsets, nbins, xy, q, k, h->stream));
    RD_HIP(hipStreamSynchronize(h->stream));
    return RD_OK;
}

}  // namespace rd

namespace {

rd_status upload_tables(rd_ctx* h, const rd_params& p) {
    h->vtile = vote_tile_for(p.measure);
    const size_t budget = std::min<size_t>(static_cast<size_t>(h->tune.vote_lds_kb) * 1024, vote_lds_max(h->vtile));
    if (h->tab_valid && same_params(h->tab_params, p) && h->tab_budget == budget) return RD_OK;
    build_tables(p, h->tabs, budget);
    const LevelTables& t = h->tabs;
    RD_HIP(hipMemcpyAsync(h->d_wtab, t.wtab.data(), t.wtab.size() * sizeof(uint32_t), hipMemcpyHostToDevice, h->stream));
    RD_HIP(hipMemcpyAsync(h->d_ktab, t.ktab.data(), t.ktab.size() * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
    RD_HIP(hipMemcpyAsync(h->d_thr, t.thr.data(), t.thr.size() * sizeof(uint64_t), hipMemcpyHostToDevice, h->stream));
    RD_HIP(hipStreamSynchronize(h->stream));   // the host vectors may change on the next call
    h->tab_params = p;
    h->tab_budget = budget;
    h->tab_valid = true;
    return RD_OK;
}

VoteArgs vote_args(rd_ctx* h, const rd_params& p, int nframes, int total_vtiles) {
    VoteArgs a{};
    a.frames = h->d_frames;
    a.nframes = nframes;
    a.total_vtiles = total_vtiles;
    a.rxy = h->d_rxy;
    a.rq = h->d_rq;
    a.bin_count = h->d_bin_count;
    a.lbase = h->tabs.lbase;
    a.r_step = h->tabs.rstep;
    a.nlevels = h->tabs.L;
    a.vote_threshold = p.vote_threshold;
    a.wtab = h->d_wtab;
    a.ktab = h->d_ktab;
    a.thr = h->d_thr;
    a.peaks = h->d_peaks;
    a.peak_count = h->d_counts;
    a.max_peaks = h->max_peaks;
    a.error = h->d_counts + h->max_frames + 1;
    a.tile_counter = h->d_counts + h->max_frames + 2;
    a.stats = h->d_stats;
    a.tile = vote_tile_for(p.measure);
    return a;
}

FitArgs fit_args(rd_ctx* h, const rd_params& p, int nframes, rd_ring* rings, uint32_t* counts_out) {
    FitArgs a{};
    a.frames = h->d_frames;
    a.counts_out = counts_out;
    a.error = h->d_counts + h->max_frames + 1;
    a.rxy = h->d_rxy;
    a.bin_count = h->d_bin_count;
    a.peaks = h->d_peaks;
    a.peak_count = h->d_counts;
    a.nframes = nframes;
    a.max_peaks = h->max_peaks;
    a.w = p.annulus_halfwidth;
    a.min_pts = p.min_fit_points;
    a.rings = rings;
    a.stats_in = h->d_stats;
    a.stats_out = reinterpret_cast<unsigned long long*>(h->dh_stats);
    a.nstats = NSTATS;
    return a;
}

rd_status mark(rd_ctx* h, int i) {
    if (h->mark_now) RD_HIP(hipEventRecord(h->ev[i], h->stream));
    return RD_OK;
}

// After the stream has been synchronised: add the elapsed times between the marks of a call
// that recorded them.
void collect_timing(rd_ctx* h, bool with_stencil) {
    if (!h->mark_now) return;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->ev[1], h->ev[2]) == hipSuccess) {
        h->t_ms[1] += ms;
        h->t_n[1] += 1;
    }
    if (with_stencil && hipEventElapsedTime(&ms, h->ev[0], h->ev[1]) == hipSuccess) {
        h->t_ms[0] += ms;
        h->t_n[0] += 1;
    }
    if (hipEventElapsedTime(&ms, h->ev[2], h->ev[3]) == hipSuccess) {
        h->t_ms[2] += ms;
        h->t_n[2] += 1;
    }
}

// Counters reset, then steps 3-5 (and steps 1-2 when with_stencil).  Kernels only, so the
// sequence can be captured in a graph.
rd_status enqueue(rd_ctx* h, const rd_params& p, int nframes, int dtype, int rg, bool with_stencil, int tt, int tv,
                  rd_ring* rings, uint32_t* counts_out) {
    RD_HIP(launch_zero2(h->d_counts, h->max_frames + 4, reinterpret_cast<uint32_t*>(h->d_stats), 2 * NSTATS,
                        h->stream));
    if (with_stencil) {
        RD_TRY(mark(h, 0));
        RD_HIP(launch_stencil(stencil_args(h, p, nframes, tt), dtype, rg, h->tune.stencil_tile, false, h->stream));
    }
    RD_TRY(mark(h, 1));
    VoteArgs va = vote_args(h, p, nframes, tv);
    if (tv <= ORDER_MAX) {
        // tile costs from sampled votes, then the queue order (costliest tiles first)
        TileCostArgs ta{};
        ta.frames = h->d_frames;
        ta.nframes = nframes;
        ta.rxy = h->d_rxy;
        ta.rq = h->d_rq;
        ta.bin_count = h->d_bin_count;
        ta.rbase = h->tabs.lbase;
        ta.rstep = h->tabs.rstep;
        ta.nlevels = h->tabs.L;
        ta.total_vtiles = tv;
        ta.tile = va.tile;
        ta.cost = h->d_tcost;
        ta.order = h->d_torder;
        RD_HIP(launch_tile_cost(ta, h->n_chunks, h->stream));
        va.tile_order = h->d_torder;
    }
    if (h->phase_on) {
        va.phase_clocks = h->d_phase;
        va.tile_clocks = h->trec_on ? h->d_trec : nullptr;
    }
    RD_HIP(launch_vote(va, h->tabs.lds, false, h->cus, h->stream));
    RD_TRY(mark(h, 2));
    RD_HIP(launch_fit(fit_args(h, p, nframes, rings, counts_out), FIT_GRID, h->stream));
    RD_TRY(mark(h, 3));
    return RD_OK;
}

// The pipeline on the frames described in d_frames; results in h_rings / h_counts.
rd_status run_pipeline(rd_ctx* h, const rd_params& p, int nframes, int dtype, int rg, int tt, int tv) {
    // With timing on, the first call after a reset and every eighth after it record the events;
    // they replay a second graph that holds the event records, the other calls the plain one
    // (event records cost the replay a few microseconds each).
    h->mark_now = h->timing && (h->t_calls++ & 7) == 0;
    const int gi = h->mark_now ? 1 : 0;
    const bool graph = h->tune.use_graph && h->stream != nullptr;
    if (graph) {
        GraphKey k;
        k.timing = h->mark_now;
        k.nframes = nframes;
        k.dtype = dtype;
        k.rg = rg;
        k.variant = h->tune.stencil_tile;
        k.total_tiles = tt;
        k.total_vtiles = tv;
        k.blocks = h->cus;
        k.lds = h->tabs.lds;
        k.bin_chunks = h->n_chunks;
        k.params = p;
        if (!h->gexec[gi] || !(k == h->gkey[gi])) {
            if (h->gexec[gi]) {
                (void)hipGraphExecDestroy(h->gexec[gi]);
                h->gexec[gi] = nullptr;
            }
            hipGraph_t g = nullptr;
            RD_HIP(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
            const rd_status st = enqueue(h, p, nframes, dtype, rg, true, tt, tv, h->dh_rings, h->dh_counts);
            const hipError_t e = hipStreamEndCapture(h->stream, &g);
            if (st != RD_OK || e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                h->mark_now = false;
                return st != RD_OK ? st : RD_E_DEVICE;
            }
            const hipError_t ei = hipGraphInstantiate(&h->gexec[gi], g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ei != hipSuccess) {
                h->gexec[gi] = nullptr;
                h->mark_now = false;
                return RD_E_DEVICE;
            }
            h->gkey[gi] = k;
        }
        RD_HIP(hipGraphLaunch(h->gexec[gi], h->stream));
    } else {
        RD_TRY(enqueue(h, p, nframes, dtype, rg, true, tt, tv, h->dh_rings, h->dh_counts));
    }
    RD_HIP(hipStreamSynchronize(h->stream));   // rings, counts and statistics arrive through mappings
    collect_timing(h, true);
    h->mark_now = false;
    return RD_OK;
}

void record_stats(rd_ctx* h, int nframes) {
    int64_t peaks = 0;
    for (int f = 0; f < nframes; ++f) peaks += std::min<uint32_t>(h->h_counts[f], h->max_peaks);
    int64_t ridges = 0;
    for (int i = 0; i < 64; ++i) ridges += static_cast<int64_t>(h->h_stats[8 + i]);
    h->last_stats[0] = ridges;
    h->last_stats[1] = static_cast<int64_t>(h->h_stats[0]);
    h->last_stats[2] = static_cast<int64_t>(h->h_stats[1]);
    h->last_stats[3] = static_cast<int64_t>(h->h_stats[3]);
    h->last_stats[4] = static_cast<int64_t>(h->h_stats[2]);
    h->last_stats[5] = peaks;
}

// Copies frame f's rings out of the pinned buffer (the fit kernel wrote them in (r_bin, b, a)
// order).
rd_status copy_rings(rd_ctx* h, int f, rd_ring* out, int32_t capacity, int32_t* n_rings) {
    const uint32_t np = h->h_counts[f];
    *n_rings = static_cast<int32_t>(np);
    if (np > static_cast<uint32_t>(h->max_peaks)) return RD_E_OVERFLOW;
    const rd_ring* src = h->h_rings + static_cast<int64_t>(f) * h->max_peaks;
    const uint32_t ncopy = std::min<uint32_t>(np, static_cast<uint32_t>(std::max(capacity, 0)));
    if (ncopy) std::memcpy(out, src, ncopy * sizeof(rd_ring));
    return np > ncopy ? RD_E_TRUNCATED : RD_OK;
}

rd_status bin_external(rd_ctx* h, const int32_t* xy, const int16_t* q, int64_t n, int W, int H) {
    const int nbx = (W + BIN - 1) / BIN, nby = (H + BIN - 1) / BIN;
    RD_HIP(hipMemsetAsync(h->d_bin_count, 0, static_cast<size_t>(nbx) * nby * sizeof(uint32_t), h->stream));
    RD_HIP(hipMemsetAsync(h->d_pixmask, 0, static_cast<size_t>(nbx) * nby * 8 * sizeof(uint32_t), h->stream));
    uint32_t* d_flag = h->d_counts + h->max_frames;
    RD_HIP(hipMemsetAsync(d_flag, 0, sizeof(uint32_t), h->stream));
    BinArgs b{};
    b.xy = xy;
    b.q = q;
    b.n = n;
    b.W = W;
    b.H = H;
    b.nbx = nbx;
    b.rxy = h->d_rxy;
    b.rq = h->d_rq;
    b.rk = h->d_rk;
    b.bin_count = h->d_bin_count;
    b.pixel_mask = h->d_pixmask;
    b.flags = d_flag;
    RD_HIP(launch_bin(b, h->stream));
    uint32_t flag = 0;
    RD_HIP(hipMemcpyAsync(&flag, d_flag, sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream));
    RD_HIP(hipStreamSynchronize(h->stream));
    // off the frame, a code step 1 cannot make, a pixel listed twice (more than 256 in a bin
    // implies a repeat)
    return flag ? RD_E_INVALID : RD_OK;
}

rd_status ridge_setup(rd_ctx* h, const int32_t* xy, const int16_t* q, int64_t n, int32_t W, int32_t H,
                      const rd_params* params) {
    if (!h || !params) return RD_E_INVALID;
    RD_TRY(rd_validate_params(params));
    if (n < 0 || (n > 0 && (!xy || !q))) return RD_E_INVALID;
    if (W < 32 || H < 32) return RD_E_INVALID;
    if (W > h->max_w || H > h->max_h) return RD_E_TOO_LARGE;
    RD_HIP(hipSetDevice(h->device));
    RD_TRY(upload_tables(h, *params));
    RD_TRY(bin_external(h, xy, q, n, W, H));
    FrameDesc fd{};
    fd.W = W;
    fd.H = H;
    fd.nbx = (W + BIN - 1) / BIN;
    fd.nby = (H + BIN - 1) / BIN;
    h->h_frames[0] = fd;
    assign_chunks(h, 1);
    RD_HIP(hipMemcpyAsync(h->d_frames, h->h_frames, sizeof(FrameDesc), hipMemcpyHostToDevice, h->stream));
    h->frames_dev_n = 0;                          // not a descriptor set setup_frames knows
    return RD_OK;
}

rd_status check_batch(rd_ctx* h, const rd_frame* frames, int32_t n) {
    if (!frames || n < 1) return RD_E_INVALID;
    if (n > h->max_frames) return RD_E_TOO_LARGE;
    int64_t px = 0;
    for (int i = 0; i < n; ++i) {
        RD_TRY(check_frame(h, &frames[i]));
        if (frames[i].dtype != frames[0].dtype) return RD_E_INVALID;
        px += static_cast<int64_t>(frames[i].width) * frames[i].height;
    }
    if (px > h->max_batch_px) return RD_E_TOO_LARGE;
    return RD_OK;
}

// Chunk numbering of a launch's frames for the ridge-stream kernels (h_frames filled):
// chunk0[i] = first chunk of frame i, chunk0[n] = total; uploaded next to the frame counts.
rd_status upload_chunks(rd_ctx* h, int n, int* total_chunks) {
    std::vector<uint32_t> c0(n + 1);
    int64_t tot = 0;
    for (int i = 0; i < n; ++i) {
        c0[i] = static_cast<uint32_t>(tot);
        tot += (static_cast<int64_t>(h->h_frames[i].nbx) * h->h_frames[i].nby + RIDGE_CHUNK - 1) / RIDGE_CHUNK;
    }
    c0[n] = static_cast<uint32_t>(tot);
    if (tot > h->max_chunks) return RD_E_TOO_LARGE;
    RD_HIP(hipMemcpyAsync(h->d_cmeta + h->max_frames, c0.data(), (n + 1) * sizeof(uint32_t), hipMemcpyHostToDevice,
                          h->stream));
    RD_HIP(hipStreamSynchronize(h->stream));        // c0 is a local vector
    *total_chunks = static_cast<int>(tot);
    return RD_OK;
}

RidgeCodeArgs ridge_code_args(rd_ctx* h, int n) {
    RidgeCodeArgs a{};
    a.frames = h->d_frames;
    a.nframes = n;
    a.chunk0 = h->d_cmeta + h->max_frames;
    a.cbase = h->d_cbase;
    a.frame_n = h->d_cmeta;
    a.flags = h->d_cmeta + 2 * h->max_frames + 2;
    a.rxy = h->d_rxy;
    a.rq = h->d_rq;
    a.rk = h->d_rk;
    a.bin_count = h->d_bin_count;
    a.offsets = h->d_eoff;
    return a;
}

bool valid_tuning(const rd_tuning& t) {
    return t.stencil_tile >= 0 && t.stencil_tile < STENCIL_VARIANTS && t.vote_lds_kb >= 16 &&
           t.vote_lds_kb * 1024 <= VOTE_LDS_MAX && (t.use_graph == 0 || t.use_graph == 1);
}

}  // namespace

// ------------------------------------------------------------------------------------------
extern "C" {

const char* rd_status_string(rd_status s) {
    switch (s) {
        case RD_OK: return "ok";
        case RD_E_INVALID: return "invalid argument";
        case RD_E_NOMEM: return "out of memory";
        case RD_E_DEVICE: return "device error";
        case RD_E_TOO_LARGE: return "frame or batch too large for this context";
        case RD_E_TRUNCATED: return "output truncated";
        case RD_E_OVERFLOW: return "internal capacity exceeded";
    }
    return "unknown status";
}

rd_status rd_validate_params(const rd_params* p) {
    if (!p) return RD_E_INVALID;
    if (!(p->sigma_smooth > 0.0f) || !(p->sigma_smooth <= 4.0f)) return RD_E_INVALID;
    if (!std::isfinite(p->k_threshold) || p->k_threshold > 0.0f) return RD_E_INVALID;
    if (p->r_step < 0 || p->r_step > R_STEP_MAX) return RD_E_INVALID;
    if (p->r_min < 1 || p->r_max < p->r_min || p->r_max > R_LIMIT) return RD_E_INVALID;
    const int rs = param_rstep(*p);
    const int top = p->r_min + rs * ((p->r_max - p->r_min) / rs + 1);   // the level past r_max
    // the lowest level's radius is at least 1: scores compare across levels as S / r
    if (p->r_min - rs < 1 || top > R_LIMIT + 1) return RD_E_INVALID;
    if (p->vote_threshold < 0 || p->vote_threshold > 65535) return RD_E_INVALID;
    if (!std::isfinite(p->peak_fraction) || p->peak_fraction < 0.0f) return RD_E_INVALID;
    if (!std::isfinite(p->sig_slope) || !std::isfinite(p->sig_icpt)) return RD_E_INVALID;
    if (p->sig_slope < 0.0f || !(p->sig_icpt > 0.0f)) return RD_E_INVALID;
    if (level_radius(*p, top) > K_MAX) return RD_E_INVALID;
    if (p->annulus_halfwidth < 0 || p->annulus_halfwidth > 64) return RD_E_INVALID;
    if (p->min_fit_points < 3) return RD_E_INVALID;
    if (p->measure != RD_MEASURE_RIDGE && p->measure != RD_MEASURE_EDGE) return RD_E_INVALID;
    if (p->curvature_fp32 != 0 && p->curvature_fp32 != 1) return RD_E_INVALID;
    return RD_OK;
}

rd_status rd_validate_ridges(const int32_t* xy, const int16_t* q, int64_t n, int32_t width, int32_t height) {
    if (n < 0 || (n > 0 && (!xy || !q)) || width < 1 || height < 1 || width > MAX_DIM || height > MAX_DIM)
        return RD_E_INVALID;
    std::vector<uint8_t> seen((static_cast<size_t>(width) * height + 7) / 8, 0);
    for (int64_t i = 0; i < n; ++i) {
        const int x = xy[2 * i], y = xy[2 * i + 1];
        if (x < 0 || x >= width || y < 0 || y >= height) return RD_E_INVALID;
        if (!ridge_code_ok(q[2 * i], q[2 * i + 1])) return RD_E_INVALID;
        const size_t pix = static_cast<size_t>(y) * width + x;
        if (seen[pix >> 3] & (1u << (pix & 7))) return RD_E_INVALID;
        seen[pix >> 3] |= static_cast<uint8_t>(1u << (pix & 7));
    }
    return RD_OK;
}

rd_status rd_level_tables(const rd_params* p, int32_t capacity_levels, int32_t* ktab, uint32_t* wtab,
                          uint64_t* thr) {
    RD_TRY(rd_validate_params(p));
    LevelTables t;
    build_tables(*p, t, vote_lds_max(vote_tile_for(p->measure)));
    if (capacity_levels < t.L) return RD_E_TRUNCATED;
    for (int i = 0; i < t.L; ++i) {
        if (ktab) ktab[i] = t.ktab[i];
        if (thr) thr[i] = t.thr[i];
        if (wtab)
            for (int d = 0; d <= K_MAX; ++d)
                wtab[i * (K_MAX + 1) + d] = t.wtab[static_cast<size_t>(i) * (K_MAX + 1) + d];
    }
    return RD_OK;
}

rd_status rd_create(const rd_create_info* info, rd_handle* out) {
    if (!out) return RD_E_INVALID;
    *out = nullptr;
    if (!info) return RD_E_INVALID;
    if (info->max_width < 32 || info->max_height < 32 || info->max_width > MAX_DIM || info->max_height > MAX_DIM)
        return RD_E_INVALID;
    if (info->max_peaks <= 0 || info->max_frames < 1) return RD_E_INVALID;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return RD_E_DEVICE;
    if (info->device < 0 || info->device >= ndev) return RD_E_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, info->device) != hipSuccess) return RD_E_DEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return RD_E_DEVICE;
    if (hipSetDevice(info->device) != hipSuccess) return RD_E_DEVICE;
    if (vote_prepare() != hipSuccess) return RD_E_DEVICE;

    rd_ctx* h = new (std::nothrow) rd_ctx();
    if (!h) return RD_E_NOMEM;
    h->device = info->device;
    h->stream = static_cast<hipStream_t>(info->stream);
    h->cus = prop.multiProcessorCount;
    h->max_w = info->max_width;
    h->max_h = info->max_height;
    h->max_peaks = info->max_peaks;
    h->max_frames = info->max_frames;
    const int64_t single = static_cast<int64_t>(h->max_w) * h->max_h;
    h->max_batch_px = std::max<int64_t>(info->max_batch_pixels, single);
    const int64_t bins_single = static_cast<int64_t>((h->max_w + BIN - 1) / BIN) * ((h->max_h + BIN - 1) / BIN);
    h->max_bins = std::max<int64_t>(bins_single, h->max_batch_px / (BIN * BIN) +
                                                   static_cast<int64_t>(h->max_frames) * (h->max_w / BIN + h->max_h / BIN + 1));
    const int64_t slots = h->max_bins * BIN_CAP;
    const int64_t npk = static_cast<int64_t>(h->max_frames) * h->max_peaks;
    const int64_t stage_bytes = h->max_batch_px * 4 + static_cast<int64_t>(h->max_frames) * 256;
    bool ok = true;
    ok = ok && hipMalloc(&h->d_stage, stage_bytes) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_rxy), slots * 4) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_rq), slots * 4) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_rk), slots * 4) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_bin_count), h->max_bins * 4) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_peaks), npk * sizeof(Peak)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_counts), (h->max_frames + 4) * sizeof(uint32_t)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_stats), NSTATS * sizeof(uint64_t)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_frames), h->max_frames * sizeof(FrameDesc)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_wtab), (R_LIMIT + 3) * (K_MAX + 1) * sizeof(uint32_t)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_ktab), (R_LIMIT + 3) * sizeof(int32_t)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_thr), (R_LIMIT + 3) * sizeof(uint64_t)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_offsets), bins_single * sizeof(int64_t)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_pixmask), bins_single * 8 * sizeof(uint32_t)) == hipSuccess;
    h->max_chunks = h->max_bins / RIDGE_CHUNK + h->max_frames + 1;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_cbase), h->max_chunks * sizeof(uint32_t)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_cmeta), (2 * h->max_frames + 4) * sizeof(uint32_t)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_eoff), (h->max_frames + 1) * sizeof(int64_t)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_tcost), ORDER_MAX * sizeof(uint32_t)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_torder), ORDER_MAX * sizeof(uint32_t)) == hipSuccess;
    ok = ok && hipMemset(h->d_tcost, 0, ORDER_MAX * sizeof(uint32_t)) == hipSuccess;   // kept zero between launches
    ok = ok && hipHostMalloc(reinterpret_cast<void**>(&h->h_rings), npk * sizeof(rd_ring), hipHostMallocMapped) == hipSuccess;
    ok = ok && hipHostMalloc(reinterpret_cast<void**>(&h->h_counts), (h->max_frames + 4) * sizeof(uint32_t),
                             hipHostMallocMapped) == hipSuccess;
    ok = ok && hipHostMalloc(reinterpret_cast<void**>(&h->h_frames), h->max_frames * sizeof(FrameDesc)) == hipSuccess;
    ok = ok && hipHostMalloc(reinterpret_cast<void**>(&h->h_stats), NSTATS * sizeof(uint64_t), hipHostMallocMapped) ==
                   hipSuccess;
    ok = ok && hipHostGetDevicePointer(reinterpret_cast<void**>(&h->dh_stats), h->h_stats, 0) == hipSuccess;
    ok = ok && hipHostGetDevicePointer(reinterpret_cast<void**>(&h->dh_rings), h->h_rings, 0) == hipSuccess;
    ok = ok && hipHostGetDevicePointer(reinterpret_cast<void**>(&h->dh_counts), h->h_counts, 0) == hipSuccess;
    if (!ok) {
        rd_destroy(h);
        return RD_E_NOMEM;
    }
    *out = h;
    return RD_OK;
}

void rd_destroy(rd_handle h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    for (hipGraphExec_t& g : h->gexec)
        if (g) (void)hipGraphExecDestroy(g);
    soft_state_free(h->soft);
    (void)hipFree(h->d_stage);
    (void)hipFree(h->d_rxy);
    (void)hipFree(h->d_rq);
    (void)hipFree(h->d_rk);
    (void)hipFree(h->d_bin_count);
    (void)hipFree(h->d_peaks);
    (void)hipFree(h->d_counts);
    (void)hipFree(h->d_stats);
    (void)hipFree(h->d_frames);
    (void)hipFree(h->d_wtab);
    (void)hipFree(h->d_ktab);
    (void)hipFree(h->d_thr);
    (void)hipFree(h->d_offsets);
    (void)hipFree(h->d_pixmask);
    (void)hipFree(h->d_cbase);
    (void)hipFree(h->d_cmeta);
    (void)hipFree(h->d_eoff);
    (void)hipFree(h->d_tcost);
    (void)hipFree(h->d_phase);
    (void)hipFree(h->d_trec);
    (void)hipFree(h->d_torder);
    for (hipEvent_t& e : h->ev)
        if (e) (void)hipEventDestroy(e);
    if (h->h_rings) (void)hipHostFree(h->h_rings);
    if (h->h_counts) (void)hipHostFree(h->h_counts);
    if (h->h_frames) (void)hipHostFree(h->h_frames);
    if (h->h_stats) (void)hipHostFree(h->h_stats);
    delete h;
}

rd_status rd_detect(rd_handle h, const rd_frame* frame, const rd_params* params, rd_ring* out, int32_t capacity,
                    int32_t* n_rings) {
    if (!h || !params || !n_rings || capacity < 0 || (capacity > 0 && !out)) return RD_E_INVALID;
    *n_rings = 0;
    RD_TRY(rd_validate_params(params));
    RD_TRY(check_frame(h, frame));
    RD_HIP(hipSetDevice(h->device));
    RD_TRY(upload_tables(h, *params));
    const int rg = gauss_radius(params->sigma_smooth);
    int tt = 0, tv = 0;
    RD_TRY(setup_frames(h, frame, 1, rg, h->tune.stencil_tile, false, &tt, &tv));
    RD_TRY(run_pipeline(h, *params, 1, frame->dtype, rg, tt, tv));
    record_stats(h, 1);
    if (h->h_counts[1]) return RD_E_OVERFLOW;
    return copy_rings(h, 0, out, capacity, n_rings);
}

static_assert(PH_COUNT + 4 == RD_VOTE_PHASE_WORDS, "the clock words the header declares");

rd_status rd_profile_vote_phases(rd_handle h, const rd_frame* frame, const rd_params* params, uint64_t* clocks) {
    if (!h || !clocks) return RD_E_INVALID;
    RD_TRY(rd_validate_params(params));
    RD_TRY(check_frame(h, frame));
    RD_HIP(hipSetDevice(h->device));
    if (!h->d_phase)
        RD_HIP(hipMalloc(reinterpret_cast<void**>(&h->d_phase), (PH_COUNT + 4) * sizeof(unsigned long long)));
    unsigned long long init[PH_COUNT + 4] = {};
    init[PH_COUNT + 3] = ~0ull;                       // the minimum's start
    RD_HIP(hipMemcpyAsync(h->d_phase, init, sizeof(init), hipMemcpyHostToDevice, h->stream));
    // one detection, launched directly (no graph), with the profiling instance of the vote kernel
    std::vector<rd_ring> rings(static_cast<size_t>(h->max_peaks));
    int32_t n = 0;
    const bool graph = h->tune.use_graph;
    h->tune.use_graph = false;
    h->phase_on = true;
    const rd_status st = rd_detect(h, frame, params, rings.data(), h->max_peaks, &n);
    h->phase_on = false;
    h->tune.use_graph = graph;
    if (st != RD_OK && st != RD_E_TRUNCATED) return st;
    unsigned long long out[PH_COUNT + 4];
    RD_HIP(hipMemcpyAsync(out, h->d_phase, sizeof(out), hipMemcpyDeviceToHost, h->stream));
    RD_HIP(hipStreamSynchronize(h->stream));
    for (int i = 0; i < PH_COUNT + 4; ++i) clocks[i] = out[i];
    return RD_OK;
}

rd_status rd_profile_vote_tiles(rd_handle h, const rd_frame* frame, const rd_params* params, uint64_t* records,
                                int32_t capacity, int32_t* n_tiles) {
    if (!h || !n_tiles || capacity < 0 || (capacity > 0 && !records)) return RD_E_INVALID;
    *n_tiles = 0;
    RD_TRY(rd_validate_params(params));
    RD_TRY(check_frame(h, frame));
    const int tv = vote_tiles(frame->width, frame->height, vote_tile_for(params->measure));
    *n_tiles = tv;
    if (tv > capacity) return RD_E_TRUNCATED;
    RD_HIP(hipSetDevice(h->device));
    if (h->trec_cap < tv) {
        (void)hipFree(h->d_trec);
        h->d_trec = nullptr;
        h->trec_cap = 0;
        RD_HIP(hipMalloc(reinterpret_cast<void**>(&h->d_trec), static_cast<size_t>(tv) * RD_VOTE_TILE_WORDS * 8));
        h->trec_cap = tv;
    }
    uint64_t clocks[RD_VOTE_PHASE_WORDS];
    h->trec_on = true;
    const rd_status st = rd_profile_vote_phases(h, frame, params, clocks);
    h->trec_on = false;
    if (st != RD_OK) return st;
    RD_HIP(hipMemcpy(records, h->d_trec, static_cast<size_t>(tv) * RD_VOTE_TILE_WORDS * 8, hipMemcpyDeviceToHost));
    return RD_OK;
}

rd_status rd_detect_batch(rd_handle h, const rd_frame* frames, int32_t n, const rd_params* params, rd_ring* out,
                          const int64_t* out_offsets, const int32_t* capacities, int32_t* n_rings) {
    if (!h || !params || !out_offsets || !capacities || !n_rings) return RD_E_INVALID;
    RD_TRY(rd_validate_params(params));
    RD_TRY(check_batch(h, frames, n));
    for (int i = 0; i < n; ++i) {
        n_rings[i] = 0;
        if (capacities[i] < 0 || (capacities[i] > 0 && !out) || out_offsets[i] < 0) return RD_E_INVALID;
    }
    RD_HIP(hipSetDevice(h->device));
    RD_TRY(upload_tables(h, *params));
    const int rg = gauss_radius(params->sigma_smooth);
    int tt = 0, tv = 0;
    RD_TRY(setup_frames(h, frames, n, rg, h->tune.stencil_tile, false, &tt, &tv));
    RD_TRY(run_pipeline(h, *params, n, frames[0].dtype, rg, tt, tv));
    record_stats(h, n);
    if (h->h_counts[n]) return RD_E_OVERFLOW;
    rd_status result = RD_OK;
    for (int i = 0; i < n; ++i) {
        const rd_status st = copy_rings(h, i, out ? out + out_offsets[i] : nullptr, capacities[i], &n_rings[i]);
        if (st == RD_E_OVERFLOW) return st;
        if (st != RD_OK) result = st;
    }
    return result;
}

rd_status rd_set_tuning(rd_handle h, const rd_tuning* t) {
    if (!h || !t || !valid_tuning(*t)) return RD_E_INVALID;
    h->tune = *t;
    return RD_OK;
}

rd_status rd_get_tuning(rd_handle h, rd_tuning* t) {
    if (!h || !t) return RD_E_INVALID;
    *t = h->tune;
    return RD_OK;
}

rd_status rd_autotune(rd_handle h, const rd_frame* frames, int32_t n, const rd_params* params, int32_t reps,
                      rd_tuning* best) {
    if (!h || !params || reps < 1) return RD_E_INVALID;
    RD_TRY(rd_validate_params(params));
    RD_TRY(check_batch(h, frames, n));
    std::vector<int32_t> counts(n), caps(n, 0);
    std::vector<int64_t> offs(n, 0);
    const rd_tuning saved = h->tune;
    rd_tuning winner = saved;
    double best_s = 1e300;
    static const int kLds[] = {RD_VOTE_LDS_KB_MAX - 36, RD_VOTE_LDS_KB_MAX - 24, RD_VOTE_LDS_KB_MAX - 12,
                               RD_VOTE_LDS_KB_MAX};
    for (int v = 0; v < STENCIL_VARIANTS; ++v) {
        for (int kb : kLds) {
            if (kb * 1024 > VOTE_LDS_MAX) continue;
            h->tune.stencil_tile = v;
            h->tune.vote_lds_kb = kb;
            h->tune.use_graph = saved.use_graph;
            const rd_status st = rd_detect_batch(h, frames, n, params, nullptr, offs.data(), caps.data(), counts.data());
            if (st != RD_OK && st != RD_E_TRUNCATED) {
                h->tune = saved;
                return st;
            }
            const auto t0 = std::chrono::steady_clock::now();
            for (int r = 0; r < reps; ++r)
                (void)rd_detect_batch(h, frames, n, params, nullptr, offs.data(), caps.data(), counts.data());
            const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (s < best_s) {
                best_s = s;
                winner = h->tune;
            }
        }
    }
    h->tune = winner;
    if (best) *best = winner;
    return RD_OK;
}

rd_status rd_read_stats(rd_handle h, int64_t* stats6) {
    if (!h || !stats6) return RD_E_INVALID;
    for (int i = 0; i < 6; ++i) stats6[i] = h->last_stats[i];
    return RD_OK;
}

rd_status rd_enable_timing(rd_handle h, int32_t enable) {
    if (!h) return RD_E_INVALID;
    RD_HIP(hipSetDevice(h->device));
    if (enable && !h->ev[0]) {
        for (hipEvent_t& e : h->ev) RD_HIP(hipEventCreate(&e));
    }
    h->timing = enable != 0;
    return RD_OK;
}

rd_status rd_read_timing(rd_handle h, double* ms_total, int64_t* launches, int32_t reset) {
    if (!h) return RD_E_INVALID;
    if (reset) h->t_calls = 0;
    for (int i = 0; i < 3; ++i) {
        if (ms_total) ms_total[i] = h->t_ms[i];
        if (launches) launches[i] = h->t_n[i];
        if (reset) {
            h->t_ms[i] = 0.0;
            h->t_n[i] = 0;
        }
    }
    return RD_OK;
}

rd_status rd_stage_curvature(rd_handle h, const rd_frame* frame, const rd_params* params, float* k_dev,
                             int16_t* q_dev) {
    if (!h || !params || !k_dev || !q_dev) return RD_E_INVALID;
    RD_TRY(rd_validate_params(params));
    RD_TRY(check_frame(h, frame));
    RD_HIP(hipSetDevice(h->device));
    const int rg = gauss_radius(params->sigma_smooth);
    int tt = 0, tv = 0;
    RD_TRY(setup_frames(h, frame, 1, rg, 0, true, &tt, &tv));
    StencilArgs sa = stencil_args(h, *params, 1, tt);
    sa.k_dense = k_dev;
    sa.q_dense = q_dev;
    sa.ridge_total = nullptr;
    RD_HIP(launch_stencil(sa, frame->dtype, rg, 0, true, h->stream));
    RD_HIP(hipStreamSynchronize(h->stream));
    return RD_OK;
}

rd_status rd_stage_ridges(rd_handle h, const rd_frame* frame, const rd_params* params, int32_t* xy_dev,
                          int16_t* q_dev, float* k_dev, int64_t capacity, int64_t* n_ridges) {
    if (!h || !params || !n_ridges || capacity < 0) return RD_E_INVALID;
    *n_ridges = 0;
    RD_TRY(rd_validate_params(params));
    RD_TRY(check_frame(h, frame));
    RD_HIP(hipSetDevice(h->device));
    RD_TRY(find_ridges(h, frame, *params));
    return gather_ridges(h, xy_dev, q_dev, k_dev, capacity, n_ridges);
}

rd_status rd_stage_accumulate(rd_handle h, const int32_t* xy_dev, const int16_t* q_dev, int64_t n, int32_t width,
                              int32_t height, const rd_params* params, uint32_t* acc_dev, uint64_t* score_dev) {
    if (!acc_dev) return RD_E_INVALID;
    RD_TRY(ridge_setup(h, xy_dev, q_dev, n, width, height, params));
    const size_t vox = static_cast<size_t>(h->tabs.L) * width * height;
    if (score_dev) RD_HIP(hipMemsetAsync(score_dev, 0, vox * sizeof(uint64_t), h->stream));
    RD_HIP(launch_zero(h->d_counts, h->max_frames + 4, h->stream));
    VoteArgs va = vote_args(h, *params, 1, vote_tiles(width, height, h->vtile));
    va.acc_dump = acc_dev;
    va.score_dump = score_dev;
    va.stats = nullptr;
    RD_HIP(launch_vote(va, h->tabs.lds, true, h->cus, h->stream));
    uint32_t err = 0;
    RD_HIP(hipMemcpyAsync(&err, h->d_counts + h->max_frames + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream));
    RD_HIP(hipStreamSynchronize(h->stream));
    return err ? RD_E_OVERFLOW : RD_OK;
}

rd_status rd_detect_ridges(rd_handle h, const int32_t* xy_dev, const int16_t* q_dev, int64_t n, int32_t width,
                           int32_t height, const rd_params* params, rd_ring* out, int32_t capacity,
                           int32_t* n_rings) {
    if (!n_rings || capacity < 0 || (capacity > 0 && !out)) return RD_E_INVALID;
    *n_rings = 0;
    RD_TRY(ridge_setup(h, xy_dev, q_dev, n, width, height, params));
    h->mark_now = h->timing;                       // every call of this entry point is timed
    const rd_status st = enqueue(h, *params, 1, RD_F32, 0, false, 0, vote_tiles(width, height, h->vtile), h->dh_rings,
                                 h->dh_counts);
    if (st != RD_OK) {
        h->mark_now = false;
        return st;
    }
    RD_HIP(hipStreamSynchronize(h->stream));
    collect_timing(h, false);
    h->mark_now = false;
    record_stats(h, 1);
    if (h->h_counts[1]) return RD_E_OVERFLOW;
    return copy_rings(h, 0, out, capacity, n_rings);
}

rd_status rd_encode_ridges(rd_handle h, const rd_frame* frames, int32_t n, const rd_params* params, uint8_t* out_dev,
                           int64_t capacity, int64_t* offsets) {
    if (!h || !params || !offsets || capacity < 0 || (capacity > 0 && !out_dev)) return RD_E_INVALID;
    if (reinterpret_cast<uintptr_t>(out_dev) % 16 != 0) return RD_E_INVALID;
    RD_TRY(rd_validate_params(params));
    RD_TRY(check_batch(h, frames, n));
    RD_HIP(hipSetDevice(h->device));
    const int rg = gauss_radius(params->sigma_smooth);
    int tt = 0, tv = 0;
    RD_TRY(setup_frames(h, frames, n, rg, h->tune.stencil_tile, false, &tt, &tv));
    int chunks = 0;
    RD_TRY(upload_chunks(h, n, &chunks));
    StencilArgs sa = stencil_args(h, *params, n, tt);
    sa.ridge_total = nullptr;
    RD_HIP(launch_stencil(sa, frames[0].dtype, rg, h->tune.stencil_tile, false, h->stream));
    RidgeCodeArgs a = ridge_code_args(h, n);
    a.enc = out_dev;
    a.capacity = capacity;
    RD_HIP(launch_ridge_encode(a, chunks, h->stream));
    RD_HIP(hipMemcpyAsync(offsets, h->d_eoff, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, h->stream));
    RD_HIP(hipStreamSynchronize(h->stream));
    return offsets[n] > capacity ? RD_E_TRUNCATED : RD_OK;
}

rd_status rd_detect_encoded(rd_handle h, const uint8_t* enc, int32_t on_device, const int64_t* offsets, int32_t n,
                            const rd_params* params, rd_ring* out, const int64_t* out_offsets,
                            const int32_t* capacities, int32_t* n_rings) {
    if (!h || !enc || !offsets || !params || !out_offsets || !capacities || !n_rings) return RD_E_INVALID;
    if (on_device != 0 && on_device != 1) return RD_E_INVALID;
    RD_TRY(rd_validate_params(params));
    if (n < 1) return RD_E_INVALID;
    if (n > h->max_frames) return RD_E_TOO_LARGE;
    for (int i = 0; i < n; ++i) {
        n_rings[i] = 0;
        if (capacities[i] < 0 || (capacities[i] > 0 && !out) || out_offsets[i] < 0) return RD_E_INVALID;
    }
    RD_HIP(hipSetDevice(h->device));
    h->vtile = vote_tile_for(params->measure);      // the descriptors below count vote tiles of this size
    // the headers, checked on the host: magic, size, the stream long enough for its count
    std::vector<uint32_t> hdr(4 * static_cast<size_t>(n));
    for (int i = 0; i < n; ++i) {
        if (offsets[i] < 0 || offsets[i + 1] < offsets[i] || (offsets[i] - offsets[0]) % 16 != 0) return RD_E_INVALID;
        if (on_device) {
            if (reinterpret_cast<uintptr_t>(enc + offsets[i]) % 16 != 0) return RD_E_INVALID;
            if (offsets[i + 1] - offsets[i] < 16) return RD_E_INVALID;
            RD_HIP(hipMemcpyAsync(&hdr[4 * i], enc + offsets[i], 16, hipMemcpyDeviceToHost, h->stream));
        } else {
            if (offsets[i + 1] - offsets[i] < 16) return RD_E_INVALID;
            std::memcpy(&hdr[4 * i], enc + offsets[i], 16);
        }
    }
    if (on_device) RD_HIP(hipStreamSynchronize(h->stream));
    int64_t px = 0, bins = 0;
    int tv = 0;
    for (int i = 0; i < n; ++i) {
        const uint32_t* hd = &hdr[4 * i];
        const int W = static_cast<int>(hd[1] & 0xffffu), H = static_cast<int>(hd[1] >> 16);
        if (hd[0] != RIDGE_MAGIC || hd[3] != 0u || W < 32 || H < 32) return RD_E_INVALID;
        if (W > h->max_w || H > h->max_h) return RD_E_TOO_LARGE;
        FrameDesc fd{};
        fd.W = W;
        fd.H = H;
        fd.nbx = (W + BIN - 1) / BIN;
        fd.nby = (H + BIN - 1) / BIN;
        const int64_t nb = static_cast<int64_t>(fd.nbx) * fd.nby;
        if (static_cast<int64_t>(hd[2]) > static_cast<int64_t>(W) * H) return RD_E_INVALID;
        if (offsets[i + 1] - offsets[i] < ridge_stream_bytes(hd[2], nb)) return RD_E_INVALID;
        fd.vtile0 = tv;
        fd.bin0 = bins;
        fd.peak0 = i * h->max_peaks;
        h->h_frames[i] = fd;
        tv += vote_tiles(W, H, h->vtile);
        bins += nb;
        px += static_cast<int64_t>(W) * H;
    }
    if (px > h->max_batch_px || bins > h->max_bins) return RD_E_TOO_LARGE;
    assign_chunks(h, n);
    RD_HIP(hipMemcpyAsync(h->d_frames, h->h_frames, n * sizeof(FrameDesc), hipMemcpyHostToDevice, h->stream));
    h->frames_dev_n = 0;                               // not a descriptor set setup_frames knows
    // the streams on the device: in place, or staged in one copy
    const uint8_t* dev = enc;
    std::vector<int64_t> doff(n + 1);
    for (int i = 0; i <= n; ++i) doff[i] = on_device ? offsets[i] : offsets[i] - offsets[0];
    if (!on_device) {
        const int64_t bytes = offsets[n] - offsets[0];
        if (bytes > h->max_batch_px * 4 + static_cast<int64_t>(h->max_frames) * 256) return RD_E_TOO_LARGE;
        RD_HIP(hipMemcpyAsync(h->d_stage, enc + offsets[0], bytes, hipMemcpyHostToDevice, h->stream));
        dev = static_cast<const uint8_t*>(h->d_stage);
    }
    RD_HIP(hipMemcpyAsync(h->d_eoff, doff.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, h->stream));
    int chunks = 0;
    RD_TRY(upload_chunks(h, n, &chunks));              // synchronises: doff is uploaded by then
    RD_TRY(upload_tables(h, *params));
    RidgeCodeArgs a = ridge_code_args(h, n);
    a.enc = const_cast<uint8_t*>(dev);
    RD_HIP(launch_zero(a.flags, 1, h->stream));
    RD_HIP(launch_ridge_decode(a, chunks, h->stream));
    uint32_t flag = 0;
    RD_HIP(hipMemcpyAsync(&flag, a.flags, sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream));
    RD_HIP(hipStreamSynchronize(h->stream));
    if (flag) return RD_E_INVALID;
    h->mark_now = h->timing;
    const rd_status st = enqueue(h, *params, n, RD_F32, 0, false, 0, tv, h->dh_rings, h->dh_counts);
    if (st != RD_OK) {
        h->mark_now = false;
        return st;
    }
    RD_HIP(hipStreamSynchronize(h->stream));
    collect_timing(h, false);
    h->mark_now = false;
    record_stats(h, n);
    if (h->h_counts[n]) return RD_E_OVERFLOW;
    rd_status result = RD_OK;
    for (int i = 0; i < n; ++i) {
        const rd_status r = copy_rings(h, i, out ? out + out_offsets[i] : nullptr, capacities[i], &n_rings[i]);
        if (r == RD_E_OVERFLOW) return r;
        if (r != RD_OK) result = r;
    }
    return result;
}

}  // extern "C"
