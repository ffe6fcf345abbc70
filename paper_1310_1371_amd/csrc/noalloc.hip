// rd_detect without a context and without any allocation: every device buffer the pipeline
// needs between its kernels lives in one static device array per GPU.
//
// The kernels are the ones rd_detect launches (ridge kernel, vote / smoothing / peak kernel,
// fit kernel) with the default tuning, so the ring list is the same, bit for bit.  The array
// is addressed only through the pointer hipGetSymbolAddress returns for the current device:
// in host code its name is a host-side stand-in, not a device address.
#include <mutex>

#include "rd_host.h"

namespace rd {
namespace {

constexpr int64_t align256(int64_t n) { return (n + 255) / 256 * 256; }

// layout of the array (byte offsets, each 256-aligned)
constexpr int64_t NA_BINS = static_cast<int64_t>(RD_NOALLOC_MAX_DIM / BIN) * (RD_NOALLOC_MAX_DIM / BIN);
constexpr int64_t NA_SLOTS = NA_BINS * BIN_CAP;
constexpr int64_t OFF_RXY = 0;
constexpr int64_t OFF_RQ = OFF_RXY + align256(NA_SLOTS * 4);
constexpr int64_t OFF_RK = OFF_RQ + align256(NA_SLOTS * 4);
constexpr int64_t OFF_BINS = OFF_RK + align256(NA_SLOTS * 4);
constexpr int64_t OFF_PEAKS = OFF_BINS + align256(NA_BINS * 4);
constexpr int64_t OFF_RINGS = OFF_PEAKS + align256(static_cast<int64_t>(RD_NOALLOC_MAX_PEAKS) * sizeof(Peak));
constexpr int64_t OFF_COUNTS = OFF_RINGS + align256(static_cast<int64_t>(RD_NOALLOC_MAX_PEAKS) * sizeof(rd_ring));
constexpr int64_t OFF_COUNTS_OUT = OFF_COUNTS + 256;
constexpr int64_t OFF_FRAME = OFF_COUNTS_OUT + 256;
constexpr int64_t OFF_WTAB = OFF_FRAME + align256(sizeof(FrameDesc));
constexpr int64_t OFF_KTAB = OFF_WTAB + align256((R_LIMIT + 3) * (K_MAX + 1) * 4);
constexpr int64_t OFF_THR = OFF_KTAB + align256((R_LIMIT + 3) * 4);
constexpr int64_t NA_TOTAL = OFF_THR + align256((R_LIMIT + 3) * 8);
static_assert(NA_TOTAL <= RD_NOALLOC_SCRATCH_BYTES, "the layout must fit the declared size");

// d_counts words as the kernels of a one-frame launch use them: [0] peaks of the frame,
// [1] (unused here: ridge-list bin overflow), [2] vote error flag, [3] vote tile queue
constexpr int NCOUNTS = 8;

static __device__ __align__(256) unsigned char scratch[RD_NOALLOC_SCRATCH_BYTES];

// per device: the array's device address and the launch facts, set once with that device
// current
constexpr int MAX_DEVICES = 64;
struct DeviceState {
    unsigned char* ptr = nullptr;
    int cus = 0;
    bool ready = false;
};
std::mutex g_mutex;
DeviceState g_state[MAX_DEVICES];

rd_status device_state(int dev, DeviceState* out) {
    if (dev < 0 || dev >= MAX_DEVICES) return RD_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_mutex);
    DeviceState& s = g_state[dev];
    if (!s.ready) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return RD_E_DEVICE;
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return RD_E_DEVICE;
        if (vote_prepare() != hipSuccess) return RD_E_DEVICE;
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return RD_E_DEVICE;
        s.ptr = static_cast<unsigned char*>(p);
        s.cus = prop.multiProcessorCount;
        s.ready = true;
    }
    *out = s;
    return RD_OK;
}

}  // namespace
}  // namespace rd

using namespace rd;

extern "C" rd_status rd_detect_noalloc(const rd_frame* frame, const rd_params* params, void* stream,
                                       rd_ring* out_dev, int32_t capacity, int32_t* n_rings) {
    if (!params || !n_rings || capacity < 0 || (capacity > 0 && !out_dev)) return RD_E_INVALID;
    *n_rings = 0;
    RD_TRY(rd_validate_params(params));
    if (!frame || !frame->data || frame->on_device != 1) return RD_E_INVALID;
    if (frame->dtype != RD_U16 && frame->dtype != RD_F32) return RD_E_INVALID;
    if (frame->width < 32 || frame->height < 32) return RD_E_INVALID;
    const int64_t esz = frame->dtype == RD_U16 ? 2 : 4;
    if (frame->pitch_bytes < frame->width * esz || frame->pitch_bytes % esz != 0) return RD_E_INVALID;
    if (frame->width > RD_NOALLOC_MAX_DIM || frame->height > RD_NOALLOC_MAX_DIM) return RD_E_TOO_LARGE;

    int dev = 0;
    RD_HIP(hipGetDevice(&dev));
    DeviceState ds;
    RD_TRY(device_state(dev, &ds));
    unsigned char* const base = ds.ptr;
    hipStream_t s = static_cast<hipStream_t>(stream);

    // host-side tables and descriptor (stack only); the copies complete before the call returns
    FixedTables tabs;
    build_fixed_tables(*params, tabs, vote_lds_max(vote_tile_for(params->measure)));
    const int W = frame->width, H = frame->height;
    const int rg = gauss_radius(params->sigma_smooth);
    int tw = 0, th = 0;
    stencil_tile_dims(0, rg, false, &tw, &th);
    FrameDesc fd{};
    fd.img = frame->data;
    fd.pitch = frame->pitch_bytes;
    fd.W = W;
    fd.H = H;
    fd.nbx = (W + BIN - 1) / BIN;
    fd.nby = (H + BIN - 1) / BIN;
    const int tt = ((W + tw - 1) / tw) * ((H + th - 1) / th);
    const int tv = vote_tiles(W, H, vote_tile_for(params->measure));

    FrameDesc* d_frame = reinterpret_cast<FrameDesc*>(base + OFF_FRAME);
    uint32_t* d_wtab = reinterpret_cast<uint32_t*>(base + OFF_WTAB);
    int32_t* d_ktab = reinterpret_cast<int32_t*>(base + OFF_KTAB);
    uint64_t* d_thr = reinterpret_cast<uint64_t*>(base + OFF_THR);
    uint32_t* d_rxy = reinterpret_cast<uint32_t*>(base + OFF_RXY);
    uint32_t* d_rq = reinterpret_cast<uint32_t*>(base + OFF_RQ);
    float* d_rk = reinterpret_cast<float*>(base + OFF_RK);
    uint32_t* d_bins = reinterpret_cast<uint32_t*>(base + OFF_BINS);
    Peak* d_peaks = reinterpret_cast<Peak*>(base + OFF_PEAKS);
    rd_ring* d_rings = reinterpret_cast<rd_ring*>(base + OFF_RINGS);
    uint32_t* d_counts = reinterpret_cast<uint32_t*>(base + OFF_COUNTS);
    uint32_t* d_counts_out = reinterpret_cast<uint32_t*>(base + OFF_COUNTS_OUT);

    RD_HIP(hipMemcpyAsync(d_frame, &fd, sizeof(FrameDesc), hipMemcpyHostToDevice, s));
    RD_HIP(hipMemcpyAsync(d_wtab, tabs.wtab, static_cast<size_t>(tabs.L) * (K_MAX + 1) * sizeof(uint32_t),
                          hipMemcpyHostToDevice, s));
    RD_HIP(hipMemcpyAsync(d_ktab, tabs.ktab, tabs.L * sizeof(int32_t), hipMemcpyHostToDevice, s));
    RD_HIP(hipMemcpyAsync(d_thr, tabs.thr, tabs.L * sizeof(uint64_t), hipMemcpyHostToDevice, s));

    // what the kernels read before writing: the peak count, the error flag and the tile
    // queue (the bin counts are written for every bin of the frame by the ridge kernel)
    RD_HIP(launch_zero(d_counts, NCOUNTS, s));

    StencilArgs sa = stencil_args_for(*params, d_frame, 1, tt);
    sa.rxy = d_rxy;
    sa.rq = d_rq;
    sa.rk = d_rk;
    sa.bin_count = d_bins;
    sa.ridge_total = nullptr;
    RD_HIP(launch_stencil(sa, frame->dtype, rg, 0, false, s));

    VoteArgs va{};
    va.frames = d_frame;
    va.nframes = 1;
    va.total_vtiles = tv;
    va.rxy = d_rxy;
    va.rq = d_rq;
    va.bin_count = d_bins;
    va.lbase = tabs.lbase;
    va.r_step = tabs.rstep;
    va.tile = vote_tile_for(params->measure);
    va.nlevels = tabs.L;
    va.vote_threshold = params->vote_threshold;
    va.wtab = d_wtab;
    va.ktab = d_ktab;
    va.thr = d_thr;
    va.peaks = d_peaks;
    va.peak_count = d_counts;
    va.max_peaks = RD_NOALLOC_MAX_PEAKS;
    va.error = d_counts + 2;
    va.tile_counter = d_counts + 3;
    va.stats = nullptr;
    RD_HIP(launch_vote(va, tabs.lds, false, ds.cus, s));

    FitArgs fa{};
    fa.frames = d_frame;
    fa.counts_out = d_counts_out;
    fa.error = d_counts + 2;
    fa.rxy = d_rxy;
    fa.bin_count = d_bins;
    fa.peaks = d_peaks;
    fa.peak_count = d_counts;
    fa.nframes = 1;
    fa.max_peaks = RD_NOALLOC_MAX_PEAKS;
    fa.w = params->annulus_halfwidth;
    fa.min_pts = params->min_fit_points;
    fa.rings = d_rings;
    fa.stats_in = nullptr;
    fa.stats_out = nullptr;
    fa.nstats = 0;
    RD_HIP(launch_fit(fa, FIT_GRID, s));

    uint32_t counts[2] = {0, 0};   // rings found, vote error flag
    RD_HIP(hipMemcpyAsync(counts, d_counts_out, sizeof(counts), hipMemcpyDeviceToHost, s));
    RD_HIP(hipStreamSynchronize(s));
    *n_rings = static_cast<int32_t>(counts[0]);
    if (counts[1] || counts[0] > static_cast<uint32_t>(RD_NOALLOC_MAX_PEAKS)) return RD_E_OVERFLOW;
    const uint32_t ncopy = counts[0] < static_cast<uint32_t>(capacity) ? counts[0] : static_cast<uint32_t>(capacity);
    if (ncopy) {
        RD_HIP(hipMemcpyAsync(out_dev, d_rings, ncopy * sizeof(rd_ring), hipMemcpyDeviceToDevice, s));
        RD_HIP(hipStreamSynchronize(s));
    }
    return counts[0] > ncopy ? RD_E_TRUNCATED : RD_OK;
}
