// Host runtime and C ABI of the ridge-directed Hough library: parameter validation, the
// per-level tables (window half-widths, fixed-point weights, score thresholds, level
// chunks), context-owned device scratch and the launch sequence of each entry point.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "rd_internal.h"

using namespace rd;

namespace {

constexpr double TWO_PI = 6.283185307179586;
constexpr double S_SCALE = 1073741824.0;   // 2^30
constexpr int CHUNK_MAX = VOTE_NLEV_MAX - 2;   // peak levels per vote work item
constexpr size_t VOTE_LDS_BUDGET = VOTE_LDS_MAX;

#define RD_HIP(call)                                   \
    do {                                               \
        if ((call) != hipSuccess) return RD_E_DEVICE;  \
    } while (0)

int gauss_radius(float sigma) { return static_cast<int>(std::ceil(4.0 * static_cast<double>(sigma))); }

double level_sigma(const rd_params& p, int r) {
    return static_cast<double>(p.sig_slope) * r + static_cast<double>(p.sig_icpt);
}

int level_radius(const rd_params& p, int r) { return static_cast<int>(std::ceil(3.0 * level_sigma(p, r))); }

// Level tables for radii r_min - 1 .. r_max + 1 (index l - (r_min - 1)).
struct LevelTables {
    int lbase = 0, L = 0;
    std::vector<uint32_t> wtab;      // L x (K_MAX + 1)
    std::vector<int32_t> ktab;       // L
    std::vector<uint64_t> thr;       // L
    std::vector<int32_t> chunks;     // chunk boundaries over r_min .. r_max + 1
    int nlev_max = 0, kmax = 0;
    size_t lds = 0;
};

void build_tables(const rd_params& p, LevelTables& t, size_t budget) {
    t.lbase = p.r_min - 1;
    t.L = p.r_max - p.r_min + 3;
    t.wtab.assign(static_cast<size_t>(t.L) * (K_MAX + 1), 0u);
    t.ktab.assign(t.L, 0);
    t.thr.assign(t.L, 0ull);
    for (int i = 0; i < t.L; ++i) {
        const int l = t.lbase + i;
        const double sg = level_sigma(p, l);
        const int K = level_radius(p, l);
        t.ktab[i] = K;
        for (int d = 0; d <= K; ++d)
            t.wtab[static_cast<size_t>(i) * (K_MAX + 1) + d] =
                static_cast<uint32_t>(std::floor(32768.0 * std::exp(-(double)(d * d) / (2.0 * sg * sg)) + 0.5));
        t.thr[i] = static_cast<uint64_t>(std::floor(static_cast<double>(p.peak_fraction) * TWO_PI * static_cast<double>(l) * S_SCALE));
    }
    // greedy level chunks: peak levels [rc0, rc1) need accumulator levels rc0-1 .. rc1
    t.chunks.clear();
    t.nlev_max = 0;
    t.kmax = 0;
    t.lds = 0;
    int rc0 = p.r_min;
    while (rc0 <= p.r_max) {
        int rc1 = rc0 + 1;
        while (rc1 <= p.r_max && rc1 + 1 - rc0 <= CHUNK_MAX &&
               vote_lds_bytes(VOTE_TILE, rc1 + 1 - rc0 + 2, t.ktab[rc1 + 1 - t.lbase]) <= budget)
            ++rc1;
        t.chunks.push_back(rc0);
        const int nlev = rc1 - rc0 + 2;
        const int kc = t.ktab[rc1 - t.lbase];
        t.lds = std::max(t.lds, vote_lds_bytes(VOTE_TILE, nlev, kc));
        t.nlev_max = std::max(t.nlev_max, nlev);
        t.kmax = std::max(t.kmax, kc);
        rc0 = rc1;
    }
    t.chunks.push_back(p.r_max + 1);
}

bool same_params(const rd_params& a, const rd_params& b) { return std::memcmp(&a, &b, sizeof(rd_params)) == 0; }

}  // namespace

struct rd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int max_w = 0, max_h = 0, max_peaks = 0, max_frames = 0;
    int64_t max_batch_px = 0;
    int64_t max_bins = 0;
    // device scratch
    void* d_stage = nullptr;            // host-frame staging, max_w * 4 bytes per row
    uint32_t* d_rxy = nullptr;
    uint32_t* d_rq = nullptr;
    float* d_rk = nullptr;
    uint32_t* d_bin_count = nullptr;
    Peak* d_peaks = nullptr;
    uint32_t* d_counts = nullptr;        // peak counts per frame + overflow flags
    rd_ring* d_rings = nullptr;
    FrameDesc* d_frames = nullptr;
    uint32_t* d_wtab = nullptr;
    int32_t* d_ktab = nullptr;
    uint64_t* d_thr = nullptr;
    int32_t* d_chunks = nullptr;
    int64_t* d_offsets = nullptr;        // stage gather offsets (per bin)
    // pinned host mirrors
    rd_ring* h_rings = nullptr;
    uint32_t* h_counts = nullptr;
    FrameDesc* h_frames = nullptr;
    // kernel timing
    bool timing = false;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    double t_ms[3] = {0, 0, 0};
    int64_t t_n[3] = {0, 0, 0};
    // level tables cache
    rd_params tab_params{};
    bool tab_valid = false;
    LevelTables tabs;
};

namespace {

rd_status check_frame(const rd_ctx* h, const rd_frame* f) {
    if (!f || !f->data) return RD_E_INVALID;
    if (f->dtype != RD_U16 && f->dtype != RD_F32) return RD_E_INVALID;
    if (f->width < 32 || f->height < 32) return RD_E_INVALID;
    const int64_t esz = f->dtype == RD_U16 ? 2 : 4;
    if (f->pitch_bytes < f->width * esz || f->pitch_bytes % esz != 0) return RD_E_INVALID;
    if (f->width > h->max_w || f->height > h->max_h) return RD_E_TOO_LARGE;
    return RD_OK;
}

rd_status upload_tables(rd_ctx* h, const rd_params& p) {
    if (h->tab_valid && same_params(h->tab_params, p)) return RD_OK;
    build_tables(p, h->tabs, VOTE_LDS_BUDGET);
    const LevelTables& t = h->tabs;
    RD_HIP(hipMemcpyAsync(h->d_wtab, t.wtab.data(), t.wtab.size() * sizeof(uint32_t), hipMemcpyHostToDevice, h->stream));
    RD_HIP(hipMemcpyAsync(h->d_ktab, t.ktab.data(), t.ktab.size() * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
    RD_HIP(hipMemcpyAsync(h->d_thr, t.thr.data(), t.thr.size() * sizeof(uint64_t), hipMemcpyHostToDevice, h->stream));
    RD_HIP(hipMemcpyAsync(h->d_chunks, t.chunks.data(), t.chunks.size() * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
    RD_HIP(hipStreamSynchronize(h->stream));   // the host vectors may change on the next call
    h->tab_params = p;
    h->tab_valid = true;
    return RD_OK;
}

// Frame descriptor of a single-frame launch (copies a host frame into the staging buffer).
rd_status prepare_single(rd_ctx* h, const rd_frame* f, int rg, FrameDesc& fd) {
    const int64_t esz = f->dtype == RD_U16 ? 2 : 4;
    fd = FrameDesc{};
    fd.W = f->width;
    fd.H = f->height;
    if (f->on_device) {
        fd.img = f->data;
        fd.pitch = f->pitch_bytes;
    } else {
        const int64_t pitch = static_cast<int64_t>(h->max_w) * 4;
        RD_HIP(hipMemcpy2DAsync(h->d_stage, pitch, f->data, f->pitch_bytes, f->width * esz, f->height,
                                hipMemcpyHostToDevice, h->stream));
        fd.img = h->d_stage;
        fd.pitch = pitch;
    }
    fd.tile0 = 0;
    fd.vtile0 = 0;
    fd.bin0 = 0;
    fd.nbx = (f->width + BIN - 1) / BIN;
    fd.nby = (f->height + BIN - 1) / BIN;
    fd.peak0 = 0;
    (void)rg;
    return RD_OK;
}

int stencil_tiles(int W, int H, int rg) {
    const int tw = stencil_tile_w(), th = stencil_tile_h(rg);
    return ((W + tw - 1) / tw) * ((H + th - 1) / th);
}

int vote_tiles(int W, int H) { return ((W + VOTE_TILE - 1) / VOTE_TILE) * ((H + VOTE_TILE - 1) / VOTE_TILE); }

StencilArgs stencil_args(rd_ctx* h, const rd_params& p, int nframes, int total_tiles) {
    StencilArgs a{};
    a.frames = h->d_frames;
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
    a.rxy = h->d_rxy;
    a.rq = h->d_rq;
    a.rk = h->d_rk;
    a.bin_count = h->d_bin_count;
    return a;
}

VoteArgs vote_args(rd_ctx* h, const rd_params& p, int nframes, int total_vtiles) {
    VoteArgs a{};
    a.frames = h->d_frames;
    a.nframes = nframes;
    a.total_vtiles = total_vtiles;
    a.nchunks = static_cast<int32_t>(h->tabs.chunks.size()) - 1;
    a.rxy = h->d_rxy;
    a.rq = h->d_rq;
    a.bin_count = h->d_bin_count;
    a.lbase = h->tabs.lbase;
    a.nlevels = h->tabs.L;
    a.vote_threshold = p.vote_threshold;
    a.chunk_start = h->d_chunks;
    a.wtab = h->d_wtab;
    a.ktab = h->d_ktab;
    a.thr = h->d_thr;
    a.peaks = h->d_peaks;
    a.peak_count = h->d_counts;
    a.max_peaks = h->max_peaks;
    a.error = h->d_counts + h->max_frames + 1;
    a.tile_counter = h->d_counts + h->max_frames + 2;
    return a;
}

FitArgs fit_args(rd_ctx* h, const rd_params& p, int nframes) {
    FitArgs a{};
    a.frames = h->d_frames;
    a.rxy = h->d_rxy;
    a.bin_count = h->d_bin_count;
    a.peaks = h->d_peaks;
    a.peak_count = h->d_counts;
    a.nframes = nframes;
    a.max_peaks = h->max_peaks;
    a.w = p.annulus_halfwidth;
    a.min_pts = p.min_fit_points;
    a.rings = h->d_rings;
    return a;
}

rd_status mark(rd_ctx* h, int i) {
    if (h->timing) RD_HIP(hipEventRecord(h->ev[i], h->stream));
    return RD_OK;
}

// Called after the stream has been synchronised: adds the elapsed times of the marks.
void collect_timing(rd_ctx* h, bool with_stencil) {
    if (!h->timing) return;
    float ms = 0.f;
    if (with_stencil && hipEventElapsedTime(&ms, h->ev[0], h->ev[1]) == hipSuccess) {
        h->t_ms[0] += ms;
        h->t_n[0] += 1;
    }
    if (hipEventElapsedTime(&ms, h->ev[1], h->ev[2]) == hipSuccess) {
        h->t_ms[1] += ms;
        h->t_n[1] += 1;
    }
    if (hipEventElapsedTime(&ms, h->ev[2], h->ev[3]) == hipSuccess) {
        h->t_ms[2] += ms;
        h->t_n[2] += 1;
    }
}

bool ring_less(const rd_ring& x, const rd_ring& y) {
    if (x.r_bin != y.r_bin) return x.r_bin < y.r_bin;
    if (x.b != y.b) return x.b < y.b;
    return x.a < y.a;
}

// Steps 3-5 of one frame whose ridges are already binned; copies the rings out.
rd_status vote_fit_collect(rd_ctx* h, const rd_params& p, FrameDesc& fd, rd_ring* out, int32_t capacity,
                           int32_t* n_rings, bool with_stencil) {
    const int nvt = vote_tiles(fd.W, fd.H);
    fd.vtile0 = 0;
    RD_HIP(hipMemsetAsync(h->d_counts, 0, sizeof(uint32_t), h->stream));
    RD_HIP(hipMemsetAsync(h->d_counts + h->max_frames + 1, 0, 2 * sizeof(uint32_t), h->stream));
    VoteArgs va = vote_args(h, p, 1, nvt);
    rd_status st = mark(h, 1);
    if (st != RD_OK) return st;
    RD_HIP(launch_vote(va, h->tabs.lds, false, h->stream));
    st = mark(h, 2);
    if (st != RD_OK) return st;
    FitArgs fa = fit_args(h, p, 1);
    RD_HIP(launch_fit(fa, 512, h->stream));
    st = mark(h, 3);
    if (st != RD_OK) return st;
    RD_HIP(hipMemcpyAsync(h->h_counts, h->d_counts, (h->max_frames + 2) * sizeof(uint32_t), hipMemcpyDeviceToHost,
                          h->stream));
    RD_HIP(hipStreamSynchronize(h->stream));
    collect_timing(h, with_stencil);
    const uint32_t np = h->h_counts[0];
    if (h->h_counts[h->max_frames + 1]) return RD_E_OVERFLOW;
    if (np > static_cast<uint32_t>(h->max_peaks)) {
        *n_rings = static_cast<int32_t>(np);
        return RD_E_OVERFLOW;
    }
    if (np) {
        RD_HIP(hipMemcpyAsync(h->h_rings, h->d_rings, np * sizeof(rd_ring), hipMemcpyDeviceToHost, h->stream));
        RD_HIP(hipStreamSynchronize(h->stream));
        std::sort(h->h_rings, h->h_rings + np, ring_less);
    }
    *n_rings = static_cast<int32_t>(np);
    const uint32_t ncopy = std::min<uint32_t>(np, static_cast<uint32_t>(std::max(capacity, 0)));
    if (ncopy) std::memcpy(out, h->h_rings, ncopy * sizeof(rd_ring));
    return np > static_cast<uint32_t>(std::max(capacity, 0)) ? RD_E_TRUNCATED : RD_OK;
}

rd_status bin_external(rd_ctx* h, const int32_t* xy, const int16_t* q, int64_t n, int W, int H) {
    const int nbx = (W + BIN - 1) / BIN, nby = (H + BIN - 1) / BIN;
    RD_HIP(hipMemsetAsync(h->d_bin_count, 0, static_cast<size_t>(nbx) * nby * sizeof(uint32_t), h->stream));
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
    b.overflow = d_flag;
    RD_HIP(launch_bin(b, h->stream));
    uint32_t* h_flag = h->h_counts + h->max_frames;
    RD_HIP(hipMemcpyAsync(h_flag, d_flag, sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream));
    RD_HIP(hipStreamSynchronize(h->stream));
    if (*h_flag & 2u) return RD_E_INVALID;
    if (*h_flag & 1u) return RD_E_OVERFLOW;
    return RD_OK;
}

rd_status ridge_setup(rd_ctx* h, const int32_t* xy, const int16_t* q, int64_t n, int32_t W, int32_t H,
                      const rd_params* params, FrameDesc& fd) {
    if (!h || !params) return RD_E_INVALID;
    rd_status st = rd_validate_params(params);
    if (st != RD_OK) return st;
    if (n < 0 || (n > 0 && (!xy || !q))) return RD_E_INVALID;
    if (W < 32 || H < 32) return RD_E_INVALID;
    if (W > h->max_w || H > h->max_h) return RD_E_TOO_LARGE;
    RD_HIP(hipSetDevice(h->device));
    st = upload_tables(h, *params);
    if (st != RD_OK) return st;
    st = bin_external(h, xy, q, n, W, H);
    if (st != RD_OK) return st;
    fd = FrameDesc{};
    fd.W = W;
    fd.H = H;
    fd.nbx = (W + BIN - 1) / BIN;
    fd.nby = (H + BIN - 1) / BIN;
    RD_HIP(hipMemcpyAsync(h->d_frames, &fd, sizeof(FrameDesc), hipMemcpyHostToDevice, h->stream));
    return RD_OK;
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
    if (p->r_min < 1 || p->r_max < p->r_min || p->r_max > R_LIMIT) return RD_E_INVALID;
    if (p->vote_threshold < 0 || p->vote_threshold > 65535) return RD_E_INVALID;
    if (!std::isfinite(p->peak_fraction) || p->peak_fraction < 0.0f) return RD_E_INVALID;
    if (!std::isfinite(p->sig_slope) || !std::isfinite(p->sig_icpt)) return RD_E_INVALID;
    if (p->sig_slope < 0.0f || !(p->sig_icpt > 0.0f)) return RD_E_INVALID;
    if (level_radius(*p, p->r_max + 1) > K_MAX) return RD_E_INVALID;
    if (p->annulus_halfwidth < 0 || p->annulus_halfwidth > 64) return RD_E_INVALID;
    if (p->min_fit_points < 3) return RD_E_INVALID;
    return RD_OK;
}

rd_status rd_level_tables(const rd_params* p, int32_t capacity_levels, int32_t* ktab, uint32_t* wtab,
                          uint64_t* thr) {
    rd_status st = rd_validate_params(p);
    if (st != RD_OK) return st;
    LevelTables t;
    build_tables(*p, t, VOTE_LDS_BUDGET);
    if (capacity_levels < t.L) return RD_E_TRUNCATED;
    for (int i = 0; i < t.L; ++i) {
        if (ktab) ktab[i] = t.ktab[i];
        if (thr) thr[i] = t.thr[i];
        if (wtab)
            for (int d = 0; d <= K_MAX; ++d) wtab[i * (K_MAX + 1) + d] = t.wtab[static_cast<size_t>(i) * (K_MAX + 1) + d];
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

    rd_ctx* h = new (std::nothrow) rd_ctx();
    if (!h) return RD_E_NOMEM;
    h->device = info->device;
    h->stream = static_cast<hipStream_t>(info->stream);
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
    bool ok = true;
    ok = ok && hipMalloc(&h->d_stage, static_cast<size_t>(single) * 4) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_rxy), slots * 4) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_rq), slots * 4) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_rk), slots * 4) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_bin_count), h->max_bins * 4) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_peaks), npk * sizeof(Peak)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_counts), (h->max_frames + 4) * sizeof(uint32_t)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_rings), npk * sizeof(rd_ring)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_frames), h->max_frames * sizeof(FrameDesc)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_wtab), (R_LIMIT + 3) * (K_MAX + 1) * sizeof(uint32_t)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_ktab), (R_LIMIT + 3) * sizeof(int32_t)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_thr), (R_LIMIT + 3) * sizeof(uint64_t)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_chunks), (R_LIMIT + 3) * sizeof(int32_t)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&h->d_offsets), bins_single * sizeof(int64_t)) == hipSuccess;
    ok = ok && hipHostMalloc(reinterpret_cast<void**>(&h->h_rings), npk * sizeof(rd_ring)) == hipSuccess;
    ok = ok && hipHostMalloc(reinterpret_cast<void**>(&h->h_counts), (h->max_frames + 4) * sizeof(uint32_t)) == hipSuccess;
    ok = ok && hipHostMalloc(reinterpret_cast<void**>(&h->h_frames), h->max_frames * sizeof(FrameDesc)) == hipSuccess;
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
    (void)hipFree(h->d_stage);
    (void)hipFree(h->d_rxy);
    (void)hipFree(h->d_rq);
    (void)hipFree(h->d_rk);
    (void)hipFree(h->d_bin_count);
    (void)hipFree(h->d_peaks);
    (void)hipFree(h->d_counts);
    (void)hipFree(h->d_rings);
    (void)hipFree(h->d_frames);
    (void)hipFree(h->d_wtab);
    (void)hipFree(h->d_ktab);
    (void)hipFree(h->d_thr);
    (void)hipFree(h->d_chunks);
    (void)hipFree(h->d_offsets);
    for (hipEvent_t& e : h->ev)
        if (e) (void)hipEventDestroy(e);
    if (h->h_rings) (void)hipHostFree(h->h_rings);
    if (h->h_counts) (void)hipHostFree(h->h_counts);
    if (h->h_frames) (void)hipHostFree(h->h_frames);
    delete h;
}

rd_status rd_detect(rd_handle h, const rd_frame* frame, const rd_params* params, rd_ring* out, int32_t capacity,
                    int32_t* n_rings) {
    if (!h || !params || !n_rings || (capacity > 0 && !out) || capacity < 0) return RD_E_INVALID;
    *n_rings = 0;
    rd_status st = rd_validate_params(params);
    if (st != RD_OK) return st;
    st = check_frame(h, frame);
    if (st != RD_OK) return st;
    RD_HIP(hipSetDevice(h->device));
    st = upload_tables(h, *params);
    if (st != RD_OK) return st;
    const int rg = gauss_radius(params->sigma_smooth);
    FrameDesc fd;
    st = prepare_single(h, frame, rg, fd);
    if (st != RD_OK) return st;
    RD_HIP(hipMemcpyAsync(h->d_frames, &fd, sizeof(FrameDesc), hipMemcpyHostToDevice, h->stream));
    const int nt = stencil_tiles(fd.W, fd.H, rg);
    StencilArgs sa = stencil_args(h, *params, 1, nt);
    st = mark(h, 0);
    if (st != RD_OK) return st;
    RD_HIP(launch_stencil(sa, frame->dtype, rg, false, h->stream));
    return vote_fit_collect(h, *params, fd, out, capacity, n_rings, true);
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
    rd_status st = rd_validate_params(params);
    if (st != RD_OK) return st;
    st = check_frame(h, frame);
    if (st != RD_OK) return st;
    RD_HIP(hipSetDevice(h->device));
    const int rg = gauss_radius(params->sigma_smooth);
    FrameDesc fd;
    st = prepare_single(h, frame, rg, fd);
    if (st != RD_OK) return st;
    RD_HIP(hipMemcpyAsync(h->d_frames, &fd, sizeof(FrameDesc), hipMemcpyHostToDevice, h->stream));
    StencilArgs sa = stencil_args(h, *params, 1, stencil_tiles(fd.W, fd.H, rg));
    sa.k_dense = k_dev;
    sa.q_dense = q_dev;
    RD_HIP(launch_stencil(sa, frame->dtype, rg, true, h->stream));
    RD_HIP(hipStreamSynchronize(h->stream));
    return RD_OK;
}

rd_status rd_stage_ridges(rd_handle h, const rd_frame* frame, const rd_params* params, int32_t* xy_dev,
                          int16_t* q_dev, float* k_dev, int64_t capacity, int64_t* n_ridges) {
    if (!h || !params || !n_ridges || capacity < 0) return RD_E_INVALID;
    *n_ridges = 0;
    rd_status st = rd_validate_params(params);
    if (st != RD_OK) return st;
    st = check_frame(h, frame);
    if (st != RD_OK) return st;
    RD_HIP(hipSetDevice(h->device));
    const int rg = gauss_radius(params->sigma_smooth);
    FrameDesc fd;
    st = prepare_single(h, frame, rg, fd);
    if (st != RD_OK) return st;
    RD_HIP(hipMemcpyAsync(h->d_frames, &fd, sizeof(FrameDesc), hipMemcpyHostToDevice, h->stream));
    StencilArgs sa = stencil_args(h, *params, 1, stencil_tiles(fd.W, fd.H, rg));
    RD_HIP(launch_stencil(sa, frame->dtype, rg, false, h->stream));
    // per-bin counts -> offsets on the host (a debug path), then one gather kernel
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
    *n_ridges = tot;
    if (tot > capacity) return RD_E_TRUNCATED;
    if (tot == 0) return RD_OK;
    RD_HIP(hipMemcpyAsync(h->d_offsets, off.data(), nbins * sizeof(int64_t), hipMemcpyHostToDevice, h->stream));
    RD_HIP(launch_gather(h->d_rxy, h->d_rq, h->d_rk, h->d_bin_count, h->d_offsets, nbins, xy_dev, q_dev, k_dev,
                            h->stream));
    RD_HIP(hipStreamSynchronize(h->stream));
    return RD_OK;
}

rd_status rd_stage_accumulate(rd_handle h, const int32_t* xy_dev, const int16_t* q_dev, int64_t n, int32_t width,
                              int32_t height, const rd_params* params, uint32_t* acc_dev, uint64_t* score_dev) {
    if (!acc_dev) return RD_E_INVALID;
    FrameDesc fd;
    rd_status st = ridge_setup(h, xy_dev, q_dev, n, width, height, params, fd);
    if (st != RD_OK) return st;
    const size_t vox = static_cast<size_t>(h->tabs.L) * width * height;
    if (score_dev) RD_HIP(hipMemsetAsync(score_dev, 0, vox * sizeof(uint64_t), h->stream));
    RD_HIP(hipMemsetAsync(h->d_counts, 0, (h->max_frames + 4) * sizeof(uint32_t), h->stream));
    VoteArgs va = vote_args(h, *params, 1, vote_tiles(width, height));
    va.acc_dump = acc_dev;
    va.score_dump = score_dev;
    RD_HIP(launch_vote(va, h->tabs.lds, true, h->stream));
    RD_HIP(hipMemcpyAsync(h->h_counts, h->d_counts, (h->max_frames + 2) * sizeof(uint32_t), hipMemcpyDeviceToHost,
                          h->stream));
    RD_HIP(hipStreamSynchronize(h->stream));
    if (h->h_counts[h->max_frames + 1]) return RD_E_OVERFLOW;
    return RD_OK;
}

rd_status rd_detect_ridges(rd_handle h, const int32_t* xy_dev, const int16_t* q_dev, int64_t n, int32_t width,
                           int32_t height, const rd_params* params, rd_ring* out, int32_t capacity,
                           int32_t* n_rings) {
    if (!n_rings || capacity < 0 || (capacity > 0 && !out)) return RD_E_INVALID;
    *n_rings = 0;
    FrameDesc fd;
    rd_status st = ridge_setup(h, xy_dev, q_dev, n, width, height, params, fd);
    if (st != RD_OK) return st;
    return vote_fit_collect(h, *params, fd, out, capacity, n_rings, false);
}

}  // extern "C"
