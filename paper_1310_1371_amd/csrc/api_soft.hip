// C ABI of the differentiable extension: ridge set with Hessians, soft accumulator and its
// adjoint, Hessian adjoint, ring-profile loss, its gradient and Levenberg-Marquardt
// refinement.  Scratch for these calls is allocated once per context, on first use, at the
// context's maximum frame size.
#include <cmath>
#include <new>

#include "rd_host.h"

using namespace rd;

namespace rd {

struct SoftState {
    int64_t max_px = 0;
    int64_t max_bins = 0;
    double* hess_planes = nullptr;    // [3][max_px] Ixx, Iyy, Ixy of one frame
    uint32_t* sxy = nullptr;          // binned soft ridges, BIN_CAP slots per bin
    double* sux = nullptr;
    double* suy = nullptr;
    float* sw = nullptr;
    uint32_t* bin_count = nullptr;
    float* planes = nullptr;          // [8][max_px]: gradient planes (3), Sobel-transposed (3), dG, temp
    uint32_t* flags = nullptr;        // [0] soft binning flags, [1] isotropic count
    uint32_t* h_flags = nullptr;      // pinned copy
};

void soft_state_free(SoftState* s) {
    if (!s) return;
    (void)hipFree(s->hess_planes);
    (void)hipFree(s->sxy);
    (void)hipFree(s->sux);
    (void)hipFree(s->suy);
    (void)hipFree(s->sw);
    (void)hipFree(s->bin_count);
    (void)hipFree(s->planes);
    (void)hipFree(s->flags);
    if (s->h_flags) (void)hipHostFree(s->h_flags);
    delete s;
}

}  // namespace rd

namespace {

constexpr double SOBEL_S5[5] = {1.0, 4.0, 6.0, 4.0, 1.0};
constexpr double SOBEL_D1[5] = {-1.0, -2.0, 0.0, 2.0, 1.0};
constexpr double SOBEL_D2[5] = {1.0, 0.0, -2.0, 0.0, 1.0};
constexpr double LM_LAMBDA0 = 1e-3, LM_DOWN = 1.0 / 3.0, LM_UP = 4.0;

rd_status soft_state(rd_ctx* h, SoftState** out) {
    if (!h->soft) {
        SoftState* s = new (std::nothrow) SoftState();
        if (!s) return RD_E_NOMEM;
        s->max_px = static_cast<int64_t>(h->max_w) * h->max_h;
        s->max_bins = static_cast<int64_t>((h->max_w + BIN - 1) / BIN) * ((h->max_h + BIN - 1) / BIN);
        const int64_t slots = s->max_bins * BIN_CAP;
        bool ok = true;
        ok = ok && hipMalloc(reinterpret_cast<void**>(&s->hess_planes), 3 * s->max_px * sizeof(double)) == hipSuccess;
        ok = ok && hipMalloc(reinterpret_cast<void**>(&s->sxy), slots * sizeof(uint32_t)) == hipSuccess;
        ok = ok && hipMalloc(reinterpret_cast<void**>(&s->sux), slots * sizeof(double)) == hipSuccess;
        ok = ok && hipMalloc(reinterpret_cast<void**>(&s->suy), slots * sizeof(double)) == hipSuccess;
        ok = ok && hipMalloc(reinterpret_cast<void**>(&s->sw), slots * sizeof(float)) == hipSuccess;
        ok = ok && hipMalloc(reinterpret_cast<void**>(&s->bin_count), s->max_bins * sizeof(uint32_t)) == hipSuccess;
        ok = ok && hipMalloc(reinterpret_cast<void**>(&s->planes), 8 * s->max_px * sizeof(float)) == hipSuccess;
        ok = ok && hipMalloc(reinterpret_cast<void**>(&s->flags), 4 * sizeof(uint32_t)) == hipSuccess;
        ok = ok && hipHostMalloc(reinterpret_cast<void**>(&s->h_flags), 4 * sizeof(uint32_t)) == hipSuccess;
        if (!ok) {
            soft_state_free(s);
            return RD_E_NOMEM;
        }
        h->soft = s;
    }
    *out = h->soft;
    return RD_OK;
}

rd_status check_dims(const rd_ctx* h, int32_t W, int32_t H) {
    if (W < 32 || H < 32) return RD_E_INVALID;
    if (W > h->max_w || H > h->max_h) return RD_E_TOO_LARGE;
    return RD_OK;
}

// Reads the two flag words back (synchronises the stream).
rd_status read_flags(rd_ctx* h, SoftState* s) {
    RD_HIP(hipMemcpyAsync(s->h_flags, s->flags, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream));
    RD_HIP(hipStreamSynchronize(h->stream));
    return RD_OK;
}

rd_status ring_args(rd_ctx* h, const rd_frame* frames, int32_t nframes, double s, RingArgs* a) {
    if (nframes < 1 || nframes > RING_FRAMES_MAX || !frames) return RD_E_INVALID;
    if (!(s > 0.0) || !std::isfinite(s)) return RD_E_INVALID;
    *a = RingArgs{};
    for (int i = 0; i < nframes; ++i) {
        RD_TRY(check_frame(h, &frames[i]));
        if (!frames[i].on_device) return RD_E_INVALID;
        a->frames[i].img = frames[i].data;
        a->frames[i].pitch = frames[i].pitch_bytes;
        a->frames[i].W = frames[i].width;
        a->frames[i].H = frames[i].height;
        a->frames[i].dtype = frames[i].dtype;
    }
    a->nframes = nframes;
    a->s = s;
    const double three_s = 3.0 * s;   // separate statements: no fused multiply-add
    a->halfwidth = three_s + 2.0;
    return RD_OK;
}

}  // namespace

extern "C" {

rd_status rd_soft_ridges(rd_handle h, const rd_frame* frame, const rd_params* params, int32_t* xy_dev,
                         double* hess_dev, int64_t capacity, int64_t* n_ridges) {
    if (!h || !params || !n_ridges || capacity < 0) return RD_E_INVALID;
    *n_ridges = 0;
    RD_TRY(rd_validate_params(params));
    if (params->measure != RD_MEASURE_RIDGE) return RD_E_INVALID;   // defined for directed ridges
    if (params->curvature_fp32) return RD_E_INVALID;                 // the Hessian in float64
    RD_TRY(check_frame(h, frame));
    RD_HIP(hipSetDevice(h->device));
    SoftState* s = nullptr;
    RD_TRY(soft_state(h, &s));
    RD_TRY(find_ridges(h, frame, *params));
    int64_t n = 0;
    const rd_status st = gather_ridges(h, xy_dev, nullptr, nullptr, capacity, &n);
    *n_ridges = n;
    if (st != RD_OK || n == 0 || !hess_dev) return st;
    // the Hessian planes of the same frame (dense stencil mode), then one gather
    const int rg = gauss_radius(params->sigma_smooth);
    int tt = 0, tv = 0;
    RD_TRY(setup_frames(h, frame, 1, rg, 0, true, &tt, &tv));
    StencilArgs sa = stencil_args(h, *params, 1, tt);
    sa.ridge_total = nullptr;
    sa.hess_dense = s->hess_planes;
    RD_HIP(launch_stencil(sa, frame->dtype, rg, 0, true, h->stream));
    RD_HIP(launch_hess_gather(s->hess_planes, frame->width, frame->height, xy_dev, n, hess_dev, h->stream));
    RD_HIP(hipStreamSynchronize(h->stream));
    return RD_OK;
}

}  // extern "C"

namespace {

// The parameter checks the soft accumulator and its adjoints share.
rd_status soft_params_ok(const rd_params* params, bool levels) {
    RD_TRY(rd_validate_params(params));
    if (params->measure != RD_MEASURE_RIDGE) return RD_E_INVALID;   // defined for directed ridges
    if (params->curvature_fp32) return RD_E_INVALID;                 // the Hessian in float64
    if (levels && param_rstep(*params) != 1) return RD_E_INVALID;   // levels in steps of one pixel
    return RD_OK;
}

int64_t acc_elems(const rd_params& p, int W, int H) {
    return static_cast<int64_t>(p.r_max - p.r_min + 3) * W * H;
}

// Enqueues the soft accumulator of one frame's ridges (flags are cleared and read by the caller).
rd_status soft_forward_one(rd_ctx* h, SoftState* s, const int32_t* xy_dev, const double* hess_dev, int64_t n,
                           int32_t width, int32_t height, const rd_params* params, float* acc_dev) {
    const int nbx = (width + BIN - 1) / BIN, nby = (height + BIN - 1) / BIN;
    RD_HIP(launch_fill_u32(s->bin_count, static_cast<int64_t>(nbx) * nby, h->stream));
    SoftBinArgs b{};
    b.xy = xy_dev;
    b.hess = hess_dev;
    b.n = n;
    b.W = width;
    b.H = height;
    b.nbx = nbx;
    b.sxy = s->sxy;
    b.sux = s->sux;
    b.suy = s->suy;
    b.sw = s->sw;
    b.bin_count = s->bin_count;
    b.flags = s->flags;
    RD_HIP(launch_soft_bin(b, h->stream));
    SoftFwdArgs f{};
    f.sxy = s->sxy;
    f.sux = s->sux;
    f.suy = s->suy;
    f.sw = s->sw;
    f.bin_count = s->bin_count;
    f.W = width;
    f.H = height;
    f.nbx = nbx;
    f.nby = nby;
    f.r_lo = params->r_min - 1;
    f.L = params->r_max - params->r_min + 3;
    f.acc = acc_dev;
    RD_HIP(launch_soft_forward(f, h->stream));
    return RD_OK;
}

rd_status soft_flags_status(rd_ctx* h, SoftState* s) {
    RD_TRY(read_flags(h, s));
    if (s->h_flags[0] & 2u) return RD_E_INVALID;
    if (s->h_flags[0] & 1u) return RD_E_OVERFLOW;
    return RD_OK;
}

}  // namespace

extern "C" {

rd_status rd_soft_forward(rd_handle h, const int32_t* xy_dev, const double* hess_dev, int64_t n, int32_t width,
                          int32_t height, const rd_params* params, float* acc_dev) {
    if (!h || !params || !acc_dev || n < 0 || (n > 0 && (!xy_dev || !hess_dev))) return RD_E_INVALID;
    RD_TRY(soft_params_ok(params, true));
    RD_TRY(check_dims(h, width, height));
    RD_HIP(hipSetDevice(h->device));
    SoftState* s = nullptr;
    RD_TRY(soft_state(h, &s));
    RD_HIP(launch_fill_u32(s->flags, 2, h->stream));
    RD_TRY(soft_forward_one(h, s, xy_dev, hess_dev, n, width, height, params, acc_dev));
    return soft_flags_status(h, s);
}

}  // extern "C"

namespace {

// Enqueues the soft accumulator's vector-Jacobian product for one frame's ridges.
rd_status soft_backward_one(rd_ctx* h, const int32_t* xy_dev, const double* hess_dev, int64_t n, int32_t width,
                            int32_t height, const rd_params* params, const float* grad_acc_dev, double* grad_hess_dev,
                            uint32_t* n_iso) {
    SoftBwdArgs a{};
    a.xy = xy_dev;
    a.hess = hess_dev;
    a.n = n;
    a.W = width;
    a.H = height;
    a.r_lo = params->r_min - 1;
    a.L = params->r_max - params->r_min + 3;
    a.grad_acc = grad_acc_dev;
    a.grad_hess = grad_hess_dev;
    a.n_iso = n_iso;
    RD_HIP(launch_soft_backward(a, h->stream));
    return RD_OK;
}

// Enqueues the Hessian adjoint of one frame (adds into grad_img_dev, [height][width]).
rd_status hessian_backward_one(rd_ctx* h, SoftState* s, const int32_t* xy_dev, const double* grad_hess_dev, int64_t n,
                               int32_t width, int32_t height, const rd_params* params, float* grad_img_dev) {
    const int64_t npx = static_cast<int64_t>(width) * height;
    float* P = s->planes;               // gradient w.r.t. Ixx, Iyy, Ixy
    float* T = s->planes + 3 * npx;     // after the transposed y correlations
    float* dG = s->planes + 6 * npx;    // gradient w.r.t. the smoothed image
    float* U = s->planes + 7 * npx;
    RD_HIP(launch_fill_f32(P, 3 * npx, h->stream));
    ScatterArgs sc{};
    sc.xy = xy_dev;
    sc.grad_hess = grad_hess_dev;
    sc.n = n;
    sc.W = width;
    sc.H = height;
    sc.planes = P;
    RD_HIP(launch_scatter_grad_hess(sc, h->stream));

    // Ixx = Sy_S5 Sx_D2 G / 64, Iyy = Sy_D2 Sx_S5 G / 64, Ixy = Sy_D1 Sx_D1 G / 64:
    // transpose the y correlations per component, then the x correlations summed
    AdjPassArgs a{};
    a.W = width;
    a.H = height;
    a.R = 2;
    a.ncomp = 3;
    const double* ty[3] = {SOBEL_S5, SOBEL_D2, SOBEL_D1};
    const double* tx[3] = {SOBEL_D2, SOBEL_S5, SOBEL_D1};
    for (int c = 0; c < 3; ++c) {
        a.in[c] = P + c * npx;
        a.out[c] = T + c * npx;
        for (int j = 0; j < 5; ++j) a.taps[c][j] = ty[c][j];
    }
    a.sum = 0;
    a.accumulate = 0;
    a.scale = 1.0;
    RD_HIP(launch_adj_pass(a, 1, h->stream));
    for (int c = 0; c < 3; ++c) {
        a.in[c] = T + c * npx;
        a.out[c] = c == 0 ? dG : nullptr;
        for (int j = 0; j < 5; ++j) a.taps[c][j] = tx[c][j];
    }
    a.sum = 1;
    a.scale = 1.0 / 64.0;
    RD_HIP(launch_adj_pass(a, 0, h->stream));

    // G = Sy_g Sx_g I with the normalised Gaussian taps
    const StencilArgs st = stencil_args(h, *params, 1, 0);
    const int rg = gauss_radius(params->sigma_smooth);
    AdjPassArgs g{};
    g.W = width;
    g.H = height;
    g.R = rg;
    g.ncomp = 1;
    for (int j = 0; j <= 2 * rg; ++j) g.taps[0][j] = st.g[j < rg ? rg - j : j - rg];
    g.in[0] = dG;
    g.out[0] = U;
    g.sum = 1;
    g.scale = 1.0;
    RD_HIP(launch_adj_pass(g, 1, h->stream));
    g.in[0] = U;
    g.out[0] = grad_img_dev;
    g.accumulate = 1;
    RD_HIP(launch_adj_pass(g, 0, h->stream));
    return RD_OK;
}

}  // namespace

extern "C" {

rd_status rd_soft_backward(rd_handle h, const int32_t* xy_dev, const double* hess_dev, int64_t n, int32_t width,
                           int32_t height, const rd_params* params, const float* grad_acc_dev, double* grad_hess_dev,
                           int64_t* n_isotropic) {
    if (!h || !params || n < 0 || (n > 0 && (!xy_dev || !hess_dev || !grad_acc_dev || !grad_hess_dev)))
        return RD_E_INVALID;
    RD_TRY(soft_params_ok(params, true));
    RD_TRY(check_dims(h, width, height));
    RD_HIP(hipSetDevice(h->device));
    SoftState* s = nullptr;
    RD_TRY(soft_state(h, &s));
    if (n_isotropic) RD_HIP(launch_fill_u32(s->flags + 1, 1, h->stream));
    RD_TRY(soft_backward_one(h, xy_dev, hess_dev, n, width, height, params, grad_acc_dev, grad_hess_dev,
                             n_isotropic ? s->flags + 1 : nullptr));
    if (n_isotropic) {
        RD_TRY(read_flags(h, s));
        *n_isotropic = s->h_flags[1];
    }
    return RD_OK;
}

rd_status rd_hessian_backward(rd_handle h, const int32_t* xy_dev, const double* grad_hess_dev, int64_t n,
                              int32_t width, int32_t height, const rd_params* params, float* grad_img_dev) {
    if (!h || !params || !grad_img_dev || n < 0 || (n > 0 && (!xy_dev || !grad_hess_dev))) return RD_E_INVALID;
    RD_TRY(soft_params_ok(params, false));
    RD_TRY(check_dims(h, width, height));
    RD_HIP(hipSetDevice(h->device));
    SoftState* s = nullptr;
    RD_TRY(soft_state(h, &s));
    return hessian_backward_one(h, s, xy_dev, grad_hess_dev, n, width, height, params, grad_img_dev);
}

// ---- batches of frames: the same kernels per frame, enqueued back to back with no host
// synchronisation between frames

rd_status rd_soft_ridges_batch(rd_handle h, const rd_frame* frames, int32_t nframes, const rd_params* params,
                               int32_t* xy_dev, double* hess_dev, int64_t capacity, int64_t* offsets) {
    if (!h || !params || !frames || !offsets || nframes < 1 || capacity < 0 || (capacity > 0 && !xy_dev))
        return RD_E_INVALID;
    offsets[0] = 0;
    bool truncated = false;
    for (int i = 0; i < nframes; ++i) {
        const int64_t off = offsets[i];
        const int64_t room = truncated ? 0 : (capacity > off ? capacity - off : 0);
        int64_t n = 0;
        const rd_status st = rd_soft_ridges(h, &frames[i], params, room ? xy_dev + 2 * off : nullptr,
                                            room && hess_dev ? hess_dev + 3 * off : nullptr, room, &n);
        if (st == RD_E_TRUNCATED) truncated = true;
        else if (st != RD_OK) return st;
        offsets[i + 1] = off + n;
    }
    return truncated ? RD_E_TRUNCATED : RD_OK;
}

namespace {

// Checks a batch's ridge offsets and sizes (host arrays).
rd_status batch_dims_ok(rd_ctx* h, const int64_t* offsets, const int32_t* widths, const int32_t* heights,
                        int32_t nframes) {
    if (!offsets || !widths || !heights || nframes < 1 || offsets[0] != 0) return RD_E_INVALID;
    for (int i = 0; i < nframes; ++i) {
        if (offsets[i + 1] < offsets[i]) return RD_E_INVALID;
        RD_TRY(check_dims(h, widths[i], heights[i]));
    }
    return RD_OK;
}

}  // namespace

rd_status rd_soft_forward_batch(rd_handle h, const int32_t* xy_dev, const double* hess_dev, const int64_t* offsets,
                                const int32_t* widths, const int32_t* heights, int32_t nframes, const rd_params* params,
                                float* acc_dev) {
    if (!h || !params || !acc_dev) return RD_E_INVALID;
    RD_TRY(soft_params_ok(params, true));
    RD_TRY(batch_dims_ok(h, offsets, widths, heights, nframes));
    if (offsets[nframes] > 0 && (!xy_dev || !hess_dev)) return RD_E_INVALID;
    RD_HIP(hipSetDevice(h->device));
    SoftState* s = nullptr;
    RD_TRY(soft_state(h, &s));
    RD_HIP(launch_fill_u32(s->flags, 2, h->stream));
    int64_t aoff = 0;
    for (int i = 0; i < nframes; ++i) {
        const int64_t o = offsets[i];
        RD_TRY(soft_forward_one(h, s, xy_dev + 2 * o, hess_dev + 3 * o, offsets[i + 1] - o, widths[i], heights[i],
                                params, acc_dev + aoff));
        aoff += acc_elems(*params, widths[i], heights[i]);
    }
    return soft_flags_status(h, s);
}

rd_status rd_soft_backward_batch(rd_handle h, const int32_t* xy_dev, const double* hess_dev, const int64_t* offsets,
                                 const int32_t* widths, const int32_t* heights, int32_t nframes,
                                 const rd_params* params, const float* grad_acc_dev, double* grad_hess_dev,
                                 int64_t* n_isotropic) {
    if (!h || !params || !grad_acc_dev) return RD_E_INVALID;
    RD_TRY(soft_params_ok(params, true));
    RD_TRY(batch_dims_ok(h, offsets, widths, heights, nframes));
    if (offsets[nframes] > 0 && (!xy_dev || !hess_dev || !grad_hess_dev)) return RD_E_INVALID;
    RD_HIP(hipSetDevice(h->device));
    SoftState* s = nullptr;
    RD_TRY(soft_state(h, &s));
    if (n_isotropic) RD_HIP(launch_fill_u32(s->flags + 1, 1, h->stream));
    int64_t aoff = 0;
    for (int i = 0; i < nframes; ++i) {
        const int64_t o = offsets[i];
        RD_TRY(soft_backward_one(h, xy_dev + 2 * o, hess_dev + 3 * o, offsets[i + 1] - o, widths[i], heights[i],
                                 params, grad_acc_dev + aoff, grad_hess_dev + 3 * o,
                                 n_isotropic ? s->flags + 1 : nullptr));
        aoff += acc_elems(*params, widths[i], heights[i]);
    }
    if (n_isotropic) {
        RD_TRY(read_flags(h, s));
        *n_isotropic = s->h_flags[1];
    }
    return RD_OK;
}

rd_status rd_hessian_backward_batch(rd_handle h, const int32_t* xy_dev, const double* grad_hess_dev,
                                    const int64_t* offsets, const int32_t* widths, const int32_t* heights,
                                    int32_t nframes, const rd_params* params, float* grad_img_dev) {
    if (!h || !params || !grad_img_dev) return RD_E_INVALID;
    RD_TRY(soft_params_ok(params, false));
    RD_TRY(batch_dims_ok(h, offsets, widths, heights, nframes));
    if (offsets[nframes] > 0 && (!xy_dev || !grad_hess_dev)) return RD_E_INVALID;
    RD_HIP(hipSetDevice(h->device));
    SoftState* s = nullptr;
    RD_TRY(soft_state(h, &s));
    int64_t poff = 0;
    for (int i = 0; i < nframes; ++i) {
        const int64_t o = offsets[i];
        RD_TRY(hessian_backward_one(h, s, xy_dev + 2 * o, grad_hess_dev + 3 * o, offsets[i + 1] - o, widths[i],
                                    heights[i], params, grad_img_dev + poff));
        poff += static_cast<int64_t>(widths[i]) * heights[i];
    }
    return RD_OK;
}

rd_status rd_fit_loss_batch(rd_handle h, const rd_frame* frames, int32_t nframes, const int32_t* frame_of_dev,
                            const double* theta_dev, const double* theta0_dev, int64_t m, double s, double* loss_dev,
                            double* ab_dev) {
    if (!h || m < 0 || (m > 0 && (!theta_dev || !theta0_dev || !loss_dev))) return RD_E_INVALID;
    if (nframes > 1 && m > 0 && !frame_of_dev) return RD_E_INVALID;
    RingArgs a;
    RD_TRY(ring_args(h, frames, nframes, s, &a));
    RD_HIP(hipSetDevice(h->device));
    a.frame_of = frame_of_dev;
    a.m = m;
    a.theta = theta_dev;
    a.theta0 = theta0_dev;
    a.loss = loss_dev;
    a.ab = ab_dev;
    RD_HIP(launch_fit_loss(a, false, h->stream));
    return RD_OK;
}

rd_status rd_fit_loss_backward_batch(rd_handle h, const rd_frame* frames, int32_t nframes, const int32_t* frame_of_dev,
                                     const double* theta_dev, const double* theta0_dev, int64_t m, double s,
                                     const double* grad_loss_dev, float* grad_img_dev, double* grad_theta_dev) {
    if (!h || m < 0 || (m > 0 && (!theta_dev || !theta0_dev || !grad_loss_dev || !grad_theta_dev)))
        return RD_E_INVALID;
    if (nframes > 1 && m > 0 && !frame_of_dev) return RD_E_INVALID;
    RingArgs a;
    RD_TRY(ring_args(h, frames, nframes, s, &a));
    RD_HIP(hipSetDevice(h->device));
    int64_t poff = 0;
    for (int i = 0; i < nframes; ++i) {        // the frames' gradient planes, back to back
        a.frames[i].grad_off = poff;
        poff += static_cast<int64_t>(frames[i].width) * frames[i].height;
    }
    a.frame_of = frame_of_dev;
    a.m = m;
    a.theta = theta_dev;
    a.theta0 = theta0_dev;
    a.grad_loss = grad_loss_dev;
    a.grad_img = grad_img_dev;
    a.grad_theta = grad_theta_dev;
    RD_HIP(launch_fit_loss(a, true, h->stream));
    return RD_OK;
}

rd_status rd_fit_loss(rd_handle h, const rd_frame* frame, const double* theta_dev, const double* theta0_dev, int64_t m,
                      double s, double* loss_dev, double* ab_dev) {
    if (!h || m < 0 || (m > 0 && (!theta_dev || !theta0_dev || !loss_dev))) return RD_E_INVALID;
    RingArgs a;
    RD_TRY(ring_args(h, frame, 1, s, &a));
    RD_HIP(hipSetDevice(h->device));
    a.m = m;
    a.theta = theta_dev;
    a.theta0 = theta0_dev;
    a.loss = loss_dev;
    a.ab = ab_dev;
    RD_HIP(launch_fit_loss(a, false, h->stream));
    return RD_OK;
}

rd_status rd_fit_loss_backward(rd_handle h, const rd_frame* frame, const double* theta_dev, const double* theta0_dev,
                               int64_t m, double s, const double* grad_loss_dev, float* grad_img_dev,
                               double* grad_theta_dev) {
    if (!h || m < 0 || (m > 0 && (!theta_dev || !theta0_dev || !grad_loss_dev || !grad_theta_dev)))
        return RD_E_INVALID;
    RingArgs a;
    RD_TRY(ring_args(h, frame, 1, s, &a));
    RD_HIP(hipSetDevice(h->device));
    a.m = m;
    a.theta = theta_dev;
    a.theta0 = theta0_dev;
    a.grad_loss = grad_loss_dev;
    a.grad_img = grad_img_dev;
    a.grad_theta = grad_theta_dev;
    RD_HIP(launch_fit_loss(a, true, h->stream));
    return RD_OK;
}

rd_status rd_refine(rd_handle h, const rd_frame* frames, int32_t nframes, const int32_t* frame_of_dev,
                    const double* theta0_dev, int64_t m, double s, int32_t iters, double tol, double* theta_dev,
                    double* loss_dev, int32_t* steps_dev) {
    if (!h || m < 0 || iters < 0 || !(tol >= 0.0) || (m > 0 && (!theta0_dev || !theta_dev))) return RD_E_INVALID;
    if (nframes > 1 && m > 0 && !frame_of_dev) return RD_E_INVALID;
    RingArgs a;
    RD_TRY(ring_args(h, frames, nframes, s, &a));
    RD_HIP(hipSetDevice(h->device));
    a.frame_of = frame_of_dev;
    a.m = m;
    a.theta0 = theta0_dev;
    a.theta_out = theta_dev;
    a.loss = loss_dev;
    a.iters = iters;
    a.tol = tol;
    a.steps_out = steps_dev;
    a.lam0 = LM_LAMBDA0;
    a.lam_down = LM_DOWN;
    a.lam_up = LM_UP;
    RD_HIP(launch_refine(a, h->stream));
    return RD_OK;
}

}  // extern "C"
