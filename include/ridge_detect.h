/*
 * ridge_detect.h -- C ABI of the MI355X (gfx950) ridge-directed circle Hough transform.
 *
 * The method (E. Afik, "Robust and highly performant ring detection algorithm for 3d
 * particle tracking using 2d microscope imaging", Sci. Rep. 5, 13584):
 *   1. Gaussian smoothing and 5x5 second-order Sobel derivatives; k_- = the smaller
 *      Hessian eigenvalue and X_- its eigenvector (Methods, "Algorithm implementation";
 *      SI, "Detailed algorithm", step 1).
 *   2. Ridge pixels: k_- below a threshold that is <= 0 and a local minimum along X_-
 *      (Results, "Directed ridge detection & votes collection"; SI step 2).
 *   3. Each ridge pixel votes +1 for (x, y) +/- r X_- at every radius in
 *      [r_min - 1, r_max + 1] (Results, same paragraph; SI, "Additional notes").
 *   4. Accumulators exceeding an integer threshold are smoothed within their radius level
 *      with Gaussian weights of width sigma(r) = slope r + intercept and divided by r; a
 *      voxel is a ring if that score exceeds a fraction of 2 pi and it is the maximum of
 *      its 3x3x3 box (Results, "Local maxima detection in a noisy parameter space";
 *      Methods; SI step 4).
 *   5. Ridge pixels inside an annulus around each peak are fitted by a circle for
 *      sub-pixel (cx, cy, r) (Results, "Ridge points classification"; SI step 5).
 *
 * Conventions shared by every entry point:
 *   - x = column, y = row, pixel centres at integers, (0, 0) at the top-left.
 *   - No entry point throws; every one returns an rd_status.  Parameters and sizes are
 *     validated on the host before any device work (RD_E_INVALID, RD_E_TOO_LARGE).
 *   - "device pointer" arguments are HIP device memory owned by the caller; the work is
 *     ordered on the stream given to rd_create and has completed when the call returns.
 *   - Host arrays are owned by the caller.  The context owns all of its device scratch,
 *     allocated in rd_create; no detection call allocates device memory.  (The
 *     differentiable entry points at the end allocate their own scratch once, on the first
 *     such call, and some of them return as soon as their work is enqueued; see there.)
 *   - One context per host thread; calls on one context must not overlap.
 */
#ifndef RIDGE_DETECT_H
#define RIDGE_DETECT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RD_OK = 0,
    RD_E_INVALID = 1,    /* bad parameter, null pointer, inconsistent sizes              */
    RD_E_NOMEM = 2,      /* device or pinned-host allocation failed in rd_create          */
    RD_E_DEVICE = 3,     /* no usable gfx950 device, or a HIP runtime error               */
    RD_E_TOO_LARGE = 4,  /* frame or batch larger than the maxima given to rd_create       */
    RD_E_TRUNCATED = 5,  /* output capacity too small; the count written is the required one */
    RD_E_OVERFLOW = 6    /* an internal list (the peaks of a frame, or the above-threshold
                            voxels of one tile's level chunk) overflowed; result invalid  */
} rd_status;

typedef enum { RD_U16 = 1, RD_F32 = 2 } rd_dtype;

/* One image (Results, "Problem statement": an image containing rings).  Row-major,
 * rows pitch_bytes apart.  u16 frames hold raw counts; f32 frames any real values. */
typedef struct {
    int32_t width;        /* >= 32 and <= rd_create_info.max_width                   */
    int32_t height;       /* >= 32 and <= rd_create_info.max_height                  */
    int64_t pitch_bytes;  /* >= width * element size                                 */
    int32_t dtype;        /* rd_dtype                                                */
    int32_t on_device;    /* 1: data is a device pointer; 0: host pointer (copied in) */
    const void* data;
} rd_frame;

/* Feature measure of steps 1-2 (rd_params.measure).  RD_MEASURE_RIDGE: directed ridges, the
 * smaller Hessian eigenvalue k_- and its eigenvector X_- (Results, "Directed ridge detection &
 * votes collection").  RD_MEASURE_EDGE: directed edges (SI, "Additional notes": the gradient
 * replaces the Hessian and its magnitude must be a local maximum along the gradient); the
 * measure is m = -|grad I| (first-order 5x5 Sobel / 128 on the smoothed frame) and the
 * direction the unit gradient, so that k_threshold and the strict-minimum test read
 * "|grad I| > -k_threshold and a strict maximum along the gradient".  Steps 3-5 are the same
 * for both. */
enum { RD_MEASURE_RIDGE = 0, RD_MEASURE_EDGE = 1 };

/* The method's knobs.  Limits checked by rd_validate_params are given per field. */
typedef struct {
    float sigma_smooth;       /* Gaussian scale-selection sigma, px; 0 < s <= 4 (Results,
                                 scale selection at about the outer ring's scale)          */
    float k_threshold;        /* threshold T_k <= 0 on the measure: curvature, image units /
                                 px^2 (SI step 2); with directed edges -|grad I|, units / px */
    int32_t r_min, r_max;     /* radius range, r_min <= r_max <= 126, searched in steps of r_step */
    int32_t vote_threshold;   /* integer hotspot threshold: A > vote_threshold (SI step 4) */
    float peak_fraction;      /* f: a peak needs S > f * 2 pi (SI step 4), 0 <= f          */
    float sig_slope;          /* sigma(r) = sig_slope * r + sig_icpt (Methods: 0.05, 0.25) */
    float sig_icpt;           /* slope >= 0, icpt > 0, ceil(3 sigma(r_max + 1)) <= 24      */
    int32_t annulus_halfwidth;/* w: members satisfy (r-w)^2 <= d^2 <= (r+w)^2, 0 <= w <= 64 */
    int32_t min_fit_points;   /* fewer annulus members than this: fit_ok = 0, >= 3         */
    int32_t measure;          /* RD_MEASURE_RIDGE or RD_MEASURE_EDGE; the differentiable
                                 entry points (rd_soft_*, rd_hessian_backward) take ridges only */
    int32_t r_step;           /* radius step s of the accumulator levels, 0 <= s <= 16 (0 reads
                                 as 1): level l has radius r_min - s + s l, l = 0 .. L - 1 with
                                 L = (r_max - r_min) / s + 3, so the peak levels are r_min,
                                 r_min + s, ... <= r_max with one level a step beyond each end
                                 (SI, "Additional notes": a lower resolution of the circle
                                 parameter space).  r_min - s >= 1 (every level has a radius of
                                 at least 1, as scores compare across levels as S / r) and the
                                 top level's radius <= 127.  s = 1 is the plain method.  The annulus half-width
                                 should cover half a step (w >= s / 2 + 1).  rd_soft_forward and
                                 rd_soft_backward take s = 1 only. */
    int32_t curvature_fp32;   /* 0: steps 1-2 filter in float64 (the default); 1: in float32,
                                 after the mean of each tile's input (with its halo) is taken
                                 out of its pixels, which the second derivatives cancel.  k_-
                                 then agrees with the float64 path to about 1e-6 of max|k_-|;
                                 ridge decisions within that of the threshold or of a
                                 neighbour can differ.  The differentiable entry points take
                                 0 only. */
} rd_params;

/* One detected ring.  (a, b, r_bin) is the Hough peak voxel; (cx, cy, r) the circle fit
 * (or the peak itself when fit_ok == 0); score = S at the peak (an ideal ring scores
 * about 2 pi). */
typedef struct {
    float cx, cy, r, score;
    int32_t a, b, r_bin;
    int32_t n_fit;            /* annulus members used by the fit */
    int32_t fit_ok;
} rd_ring;

typedef struct {
    int32_t device;           /* HIP device ordinal                                        */
    int32_t max_width;        /* largest frame the context accepts (<= 65535)              */
    int32_t max_height;
    int32_t max_peaks;        /* capacity of the per-frame peak list (> 0)                 */
    int32_t max_frames;       /* largest batch for rd_detect_batch (>= 1)                  */
    int64_t max_batch_pixels; /* sum of width*height over a batch (>= max_width*max_height) */
    void* stream;             /* hipStream_t the context orders its work on; NULL = default */
} rd_create_info;

typedef struct rd_ctx* rd_handle;

/* Human-readable name of a status code (static storage). */
const char* rd_status_string(rd_status s);

/* Host-only check of a parameter set; no device needed. */
rd_status rd_validate_params(const rd_params* p);

/* Host-only: the per-level tables the library derives from *p for the level radii
 * r = r_min - s + s i, i = 0 .. L - 1 (s = r_step, L = (r_max - r_min) / s + 3; caller arrays
 * of at least L entries, wtab of L * 25): ktab[i] = K(r) = ceil(3 sigma(r)),
 * sigma(r) = sig_slope r + sig_icpt in double;
 * wtab[i * 25 + d] = floor(2^15 exp(-d^2 / (2 sigma(r)^2)) + 1/2) for d <= K(r), else 0
 * (the separable fixed-point smoothing factors, Methods "Algorithm implementation");
 * thr[i] = floor(((f * 2 pi) * r) * 2^30), so that S > f 2 pi <=> S_int > thr (SI step 4).
 * Any output may be NULL. */
rd_status rd_level_tables(const rd_params* p, int32_t capacity_levels, int32_t* ktab, uint32_t* wtab,
                          uint64_t* thr);

/* Create a context on info->device; allocates all device scratch for the given maxima.
 * *out is set to NULL on failure. */
rd_status rd_create(const rd_create_info* info, rd_handle* out);

/* Free a context and its device memory.  NULL is ignored. */
void rd_destroy(rd_handle h);

/* Full pipeline on one frame.  out is a host array of `capacity` rings; *n_rings receives
 * the number of rings found, in ascending (r_bin, b, a) order.  If capacity is too small
 * the first `capacity` rings are written, *n_rings holds the full count and the call
 * returns RD_E_TRUNCATED. */
rd_status rd_detect(rd_handle h, const rd_frame* frame, const rd_params* params,
                    rd_ring* out, int32_t capacity, int32_t* n_rings);

/* ---- batches: many frames in one launch sequence ---------------------------------- */

/* The full pipeline on n frames (1 <= n <= rd_create_info.max_frames, total pixels <=
 * max_batch_pixels; all frames of one dtype; sizes may differ).  The frames are described
 * to the kernels by a device-side table; every kernel runs once for the whole batch (the
 * vote kernel's blocks are persistent and take tiles of any frame from a queue), and the
 * launch sequence is captured in a HIP graph and replayed while the batch layout (frame
 * count, tile counts, dtype, parameters' level chunks, tuning) stays the same.  Rings of
 * frame i go to out[out_offsets[i] ...] (at most capacities[i], host memory), n_rings[i]
 * receives the count (ascending (r_bin, b, a)).  Results are bit-identical to calling
 * rd_detect on each frame.  RD_E_TRUNCATED if any frame's capacity was too small. */
rd_status rd_detect_batch(rd_handle h, const rd_frame* frames, int32_t n, const rd_params* params,
                          rd_ring* out, const int64_t* out_offsets, const int32_t* capacities,
                          int32_t* n_rings);

/* Largest vote_lds_kb: what the vote kernel's own LDS leaves of a compute unit's 160 KiB. */
#define RD_VOTE_LDS_KB_MAX 89

/* Launch configuration choices.  None changes any result.  A new context starts at
 * {0, RD_VOTE_LDS_KB_MAX, 1}. */
typedef struct {
    int32_t stencil_tile;  /* ridge kernel tile: 0 = 64x32 (64x16 when ceil(4 sigma) > 8),
                              1 = 32x32, 2 = 64x16                                          */
    int32_t vote_lds_kb;   /* LDS for one tile's vote histograms, 16..RD_VOTE_LDS_KB_MAX
                              (KiB); more levels per pass with more LDS                      */
    int32_t use_graph;     /* 1: capture and replay launch sequences as HIP graphs (needs a
                              non-null stream)                                               */
} rd_tuning;

rd_status rd_set_tuning(rd_handle h, const rd_tuning* t);
rd_status rd_get_tuning(rd_handle h, rd_tuning* t);

/* Time every rd_tuning choice on the given batch (reps timed runs each, after one warm-up),
 * keep the fastest in the context and return it in *best (may be NULL). */
rd_status rd_autotune(rd_handle h, const rd_frame* frames, int32_t n, const rd_params* params,
                      int32_t reps, rd_tuning* best);

/* Counters of the last detection call (any entry point that ran the vote kernel):
 * [0] ridge pixels, [1] vote increments made in the per-tile histograms (a vote within the
 * smoothing margin of a tile border is made in every tile region that holds it), [2]
 * hotspots (A > T_int, counted once per level chunk that scores them), [3] smoothing taps
 * evaluated, [4] above-threshold voxels, [5] peaks. */
rd_status rd_read_stats(rd_handle h, int64_t* stats6);

/* ---- kernel timing (measurement) ---------------------------------------------------- */

/* Turn per-kernel timing on (1) or off (0).  When on, detection calls record HIP events on
 * the context's stream around each kernel launch (a small per-launch cost); with graphs in
 * use the records are nodes of the captured graph, so the timed calls still replay it. */
rd_status rd_enable_timing(rd_handle h, int32_t enable);

/* Accumulated kernel time since the last reset, per stage: [0] ridge kernel (steps 1-2),
 * [1] vote/smooth/peak kernel (steps 3-4), [2] fit kernel (step 5); ms_total[i] in
 * milliseconds and launches[i] the number of launches timed: the first call after a reset
 * and every eighth call after it are timed.  reset != 0 clears them. */
rd_status rd_read_timing(rd_handle h, double* ms_total, int64_t* launches, int32_t reset);

/* Measurement only: the device's rate of LDS atomic adds at random addresses, the ceiling of
 * the vote step (one LDS atomic add per vote).  Workgroups of 1024 threads with 64 KiB of u32
 * counters each add into a pseudo-random 16-bit half per iteration; with_return = 1 keeps the
 * returned old values (as the vote kernel does), 0 discards them.  *atomics_per_s receives
 * the best of three timed launches (HIP events on the null stream of `device`), *ms (may be
 * NULL) that launch's duration.  Allocates nothing; RD_E_DEVICE without a usable device. */
rd_status rd_measure_lds_atomics(int32_t device, int32_t with_return, double* atomics_per_s, double* ms);

/* Measurement only: one rd_detect of `frame`, launched directly (no graph), with a
 * profiling instance of the vote kernel (steps 3-4) that reads the shader clock after the
 * barrier ending each phase of each tile (and one barrier of its own between the 3x3x3 test
 * and the next chunk's clear).  clocks[0..7] (host) receive the clocks summed over the
 * workgroups of: tile set-up (queue, candidate bins, first histogram clear), ridge staging
 * (records, level ranges), the item sort, votes with hotspot listing, scores, the
 * above-threshold list, the 3x3x3 test with peak output, and the next level chunk's clear
 * and weight rows; clocks[8] the workgroups' summed lifetimes, clocks[9] the tiles,
 * clocks[10] and clocks[11] the longest and the shortest workgroup lifetime.  Same
 * validation as rd_detect; RD_E_OVERFLOW as rd_detect. */
#define RD_VOTE_PHASE_WORDS 12
rd_status rd_profile_vote_phases(rd_handle h, const rd_frame* frame, const rd_params* params, uint64_t* clocks);

/* Measurement only: the same profiled rd_detect, recording each vote tile of the frame.
 * records (host, 4 x capacity words) receive for vote tile t (row-major over the frame's
 * T x T tiles) at records[4 t .. 4 t + 3]: the workgroup that ran it, its position in the
 * launch's queue, the shader clock when the workgroup took it and the clock when that
 * workgroup took its next tile or ended.  Workgroups on different XCDs read different clocks,
 * so only a tile's end minus its start is meaningful.  *n_tiles receives the frame's vote
 * tiles; RD_E_TRUNCATED (nothing written) when they exceed capacity.  Same validation as
 * rd_detect; RD_E_OVERFLOW as rd_detect. */
#define RD_VOTE_TILE_WORDS 4
rd_status rd_profile_vote_tiles(rd_handle h, const rd_frame* frame, const rd_params* params, uint64_t* records,
                                int32_t capacity, int32_t* n_tiles);

/* ---- stage entry points (parity checks; same kernels as rd_detect) ------------------- */

/* Step 1 only: k_- (float, H x W, row-major, device pointer) and the direction code of
 * X_- (int16 pairs (qx, qy) per pixel, H x W x 2, device pointer).  The code is
 * rint(2^14 X_-) with qy > 0, or qy == 0 and qx > 0. */
rd_status rd_stage_curvature(rd_handle h, const rd_frame* frame, const rd_params* params,
                             float* k_dev, int16_t* q_dev);

/* Steps 1-2: the ridge list (device pointers, each sized for `capacity` ridges):
 * xy_dev = (x, y) int32 pairs, q_dev = (qx, qy) int16 pairs, k_dev = k_- as float; any of
 * the three may be NULL.  The order is grouped by 16x16 pixel bin.  *n_ridges receives
 * the count; RD_E_TRUNCATED if it exceeds capacity. */
rd_status rd_stage_ridges(rd_handle h, const rd_frame* frame, const rd_params* params,
                          int32_t* xy_dev, int16_t* q_dev, float* k_dev,
                          int64_t capacity, int64_t* n_ridges);

/* Host-only check of a ridge list (host arrays): every pixel inside the width x height frame
 * and listed once, every direction code one that step 1 produces, i.e. rint(2^14 X_-) of a
 * unit X_- in canonical sign: |qx^2 + qy^2 - 2^28| <= 2^15 and (qy > 0, or qy == 0 and
 * qx > 0).  RD_OK or RD_E_INVALID.  rd_stage_accumulate and rd_detect_ridges apply the same
 * test on the device.  These are the lists for which the integer votes are exact: a voxel at
 * level r then takes at most one vote per lattice offset that the rounded r X_- can reach
 * (about 8 r), far below the 16-bit counters and the 32-bit partial sums of the score. */
rd_status rd_validate_ridges(const int32_t* xy, const int16_t* q, int64_t n, int32_t width, int32_t height);

/* Step 3 (and the scores of step 4) from a caller-given ridge list: xy_dev = (x, y) int32
 * pairs and q_dev = (qx, qy) int16 pairs for n ridges (device pointers; the list must pass
 * the test of rd_validate_ridges, checked on the device: RD_E_INVALID otherwise; any order,
 * e.g. the bin order of rd_stage_ridges or raster order).  acc_dev receives the dense vote
 * accumulator, uint32 [L][height][width], level i at radius r_min - s + s i
 * (L = (r_max - r_min) / s + 3, s = r_step).  score_dev (may be NULL) receives the integer smoothed score
 * S_int = sum W(|dx|) W(|dy|) A (W = 15-bit fixed-point Gaussian factors) at hotspots and
 * 0 elsewhere, uint64 [L][height][width]; the score is S = S_int / (r 2^30). */
rd_status rd_stage_accumulate(rd_handle h, const int32_t* xy_dev, const int16_t* q_dev,
                              int64_t n, int32_t width, int32_t height,
                              const rd_params* params, uint32_t* acc_dev, uint64_t* score_dev);

/* Steps 3-5 from a caller-given ridge list (as rd_stage_accumulate); output as rd_detect. */
rd_status rd_detect_ridges(rd_handle h, const int32_t* xy_dev, const int16_t* q_dev,
                           int64_t n, int32_t width, int32_t height, const rd_params* params,
                           rd_ring* out, int32_t capacity, int32_t* n_rings);

/* ---- encoded ridge streams ----------------------------------------------------------------
 *
 * A frame's ridges (pixel and direction code) in a compact, self-describing byte stream that
 * stands in for the frame after step 2 (SI, "Additional notes": the ridge coordinates with
 * their directions as a compressed representation of the image; Introduction: the data
 * flow of the experiment is about 180 GB per hour).  Stream of one frame, little endian:
 *   bytes 0-15   u32 0x31524452 ("RDR1"), u16 width, u16 height, u32 ridge count n, u32 0
 *   then         u16 per 16x16 pixel bin (bins in raster order): ridges in the bin
 *   then         u8 per ridge, the ridges bin after bin: its pixel in the bin, (y & 15) << 4 | (x & 15)
 *   then         zero bytes to a multiple of 4, then u32 per ridge in the same order:
 *                qx | qy << 16 (the direction code of step 1), then zero bytes to a multiple of 16
 * About 5 bytes per ridge plus 2 per 256 pixels (a 2048^2 u16 frame of the stream workload:
 * about 1 MB against 8 MB).  Streams of a batch follow each other, each 16-byte aligned. */

/* Steps 1-2 on n frames (as rd_detect_batch takes them), then their ridges encoded into
 * out_dev (a 16-byte aligned device buffer of `capacity` bytes), frame i at byte offsets[i]
 * (host array of n + 1; offsets[n] = the total).  The ridges are those rd_detect finds.
 * RD_E_TRUNCATED if the total exceeds capacity: the offsets are still filled, and the
 * frames that do not fit are not written. */
rd_status rd_encode_ridges(rd_handle h, const rd_frame* frames, int32_t n, const rd_params* params,
                           uint8_t* out_dev, int64_t capacity, int64_t* offsets);

/* Steps 3-5 from n encoded streams: stream i at enc + offsets[i] (offsets: host array of
 * n + 1; each stream 16-byte aligned relative to offsets[0], and offsets[i + 1] - offsets[i]
 * at least its size), enc in host memory (on_device = 0, copied in) or device memory
 * (on_device = 1).  Every stream is checked: the header (magic, width and height 32 ..
 * the context's maxima, n <= width * height, the stream long enough) on the host, then on the
 * device the bin counts (each <= 256, summing to n) and every ridge: inside the frame, a
 * direction code step 1 produces (as rd_validate_ridges) and its pixel listed once;
 * RD_E_INVALID on any failure, before the votes.  Output as rd_detect_batch (rings of frame
 * i at out + out_offsets[i], at most capacities[i], n_rings[i] the count).  The rings are
 * those rd_detect_batch finds on the frames the streams were encoded from. */
rd_status rd_detect_encoded(rd_handle h, const uint8_t* enc, int32_t on_device, const int64_t* offsets, int32_t n,
                            const rd_params* params, rd_ring* out, const int64_t* out_offsets,
                            const int32_t* capacities, int32_t* n_rings);

/* ---- detection without allocation ------------------------------------------------------
 *
 * For callers that cannot allocate device memory (tight serving loops, harnesses that forbid
 * hipMalloc and friends): rd_detect on one device-resident frame with no context.  Every
 * buffer the pipeline passes between its kernels (ridge bins, peak list, counters, level
 * tables, frame descriptor, ring staging) lives in one static device array of
 * RD_NOALLOC_SCRATCH_BYTES on each GPU the call runs on, held until the process ends; the
 * call itself allocates nothing (no hipMalloc, no hipFree, no allocating library routine).
 * The kernels and the tuning are rd_detect's defaults, so the ring list is bit-identical to
 * rd_detect's on the same frame and parameters.
 *   - frame->on_device must be 1, width and height <= RD_NOALLOC_MAX_DIM (RD_E_TOO_LARGE
 *     beyond; the other frame rules as rd_detect).
 *   - The work runs on the calling thread's current device, ordered on `stream` (a
 *     hipStream_t; NULL = the default stream), and has completed when the call returns.
 *   - out_dev: a device array of `capacity` rings, written in ascending (r_bin, b, a) order;
 *     *n_rings (host) receives the count.  RD_E_TRUNCATED as rd_detect; RD_E_OVERFLOW when a
 *     frame has more than RD_NOALLOC_MAX_PEAKS peaks (or a vote tile's list overflowed).
 *   - All calls on one GPU share its array, which keeps the last call's contents: calls that
 *     overlap on one GPU (other threads, other streams) race and must be serialised by the
 *     caller. */
#define RD_NOALLOC_MAX_DIM 1024
#define RD_NOALLOC_MAX_PEAKS 8192
#define RD_NOALLOC_SCRATCH_BYTES (13 * 1024 * 1024)
rd_status rd_detect_noalloc(const rd_frame* frame, const rd_params* params, void* stream,
                            rd_ring* out_dev, int32_t capacity, int32_t* n_rings);

/* ---- differentiable extension ------------------------------------------------------------
 *
 * The paper's votes are integer and its ridge selection is a threshold, so nothing of
 * steps 3-5 is differentiable.  These calls relax the vote onto the same ridge set and the
 * same Hessian (step 1) and fit a ring-intensity profile, with hand-written adjoints:
 *
 *   soft accumulator  A~_r(c) = sum over ridges p, s = +-1 of w_p beta(p + s r u_p - c),
 *                     beta(d) = max(0, 1 - |dx|) max(0, 1 - |dy|), w_p = -k_-(p), u_p the
 *                     unit eigenvector X_-(p) (continuous, not the step-3 code), radii
 *                     r_min - 1 .. r_max + 1 as the votes; cells off the frame are dropped.
 *   ring fit loss     L_j = sum over the window W_j of (I(p) - B_j - A_j g_j(p))^2 with
 *                     g_j(p) = exp(-(|p - c_j| - r_j)^2 / (2 s^2)); (A_j, B_j) are the
 *                     least-squares fit at the current ring (c_j, r_j) and
 *                     W_j = {p : | |p - c0_j| - r0_j | <= 3 s + 2} is fixed by a starting
 *                     ring (c0_j, r0_j).  The circles of step 5 are the usual start.
 *
 * Conventions of this section: all pointers are device pointers owned by the caller;
 * ring parameters theta are float64 triples (cx, cy, r); the first call of this section on a
 * context allocates its scratch (about 24 + 100 bytes per pixel of the context's maximum
 * frame) and returns RD_E_NOMEM if that fails.  Calls that say "enqueued" return once their
 * kernels are queued on the context's stream; the others return with the work complete.
 */

/* The ridge set of step 2 (as rd_stage_ridges, bin order) and the Hessian of step 1 at each
 * ridge pixel: xy_dev int32 (x, y) pairs and hess_dev float64 (Ixx, Iyy, Ixy) triples, each
 * sized for `capacity` ridges (hess_dev may be NULL).  RD_E_TRUNCATED if the count, written
 * to *n_ridges, exceeds capacity. */
rd_status rd_soft_ridges(rd_handle h, const rd_frame* frame, const rd_params* params,
                         int32_t* xy_dev, double* hess_dev, int64_t capacity, int64_t* n_ridges);

/* The soft accumulator of n ridges (xy_dev, hess_dev as rd_soft_ridges gives them) into
 * acc_dev, float32 [L][height][width], L = r_max - r_min + 3; every element is written.
 * RD_E_INVALID if a ridge lies off the frame, RD_E_OVERFLOW if more than 256 ridges fall in
 * one 16x16 pixel bin (only possible with duplicates). */
rd_status rd_soft_forward(rd_handle h, const int32_t* xy_dev, const double* hess_dev, int64_t n,
                          int32_t width, int32_t height, const rd_params* params, float* acc_dev);

/* Vector-Jacobian product of rd_soft_forward: given grad_acc_dev = dL/dA~ (float32, shape of
 * acc_dev), writes grad_hess_dev = dL/d(Ixx, Iyy, Ixy) per ridge (float64 triples).  Through
 * k_- = X_-^T H X_- and dX_- = (X_+^T dH X_- / (k_- - k_+)) X_+; where the eigenvalues
 * nearly coincide (|k_+ - k_-| / 2 <= 1e-12 max|H|) the X_- term is dropped and counted in
 * *n_isotropic (may be NULL: then the call is enqueued). */
rd_status rd_soft_backward(rd_handle h, const int32_t* xy_dev, const double* hess_dev, int64_t n,
                           int32_t width, int32_t height, const rd_params* params,
                           const float* grad_acc_dev, double* grad_hess_dev, int64_t* n_isotropic);

/* Adjoint of step 1's Hessian (Gaussian smoothing, then the 5x5 second-order Sobel kernels
 * / 64, each 1D pass with reflect-101 borders) applied to per-ridge gradients grad_hess_dev
 * (float64 triples at xy_dev): ADDS dL/dI into grad_img_dev, float32 [height][width]
 * contiguous.  The reflect-101 halo is folded back onto the mirrored pixels.  Enqueued. */
rd_status rd_hessian_backward(rd_handle h, const int32_t* xy_dev, const double* grad_hess_dev,
                              int64_t n, int32_t width, int32_t height, const rd_params* params,
                              float* grad_img_dev);

/* Ring fit loss of m rings on one frame (device frame, u16 or f32): loss_dev[j] = L_j
 * (float64) and, if ab_dev is not NULL, ab_dev[2j..2j+1] = (A_j, B_j).  s > 0 is the
 * profile width in pixels.  An empty window gives L = 0, A = B = 0; a window where the
 * profile is constant gives A = 0, B = mean.  Enqueued. */
rd_status rd_fit_loss(rd_handle h, const rd_frame* frame, const double* theta_dev,
                      const double* theta0_dev, int64_t m, double s, double* loss_dev,
                      double* ab_dev);

/* Gradient of sum_j grad_loss_dev[j] L_j: ADDS d/dI into grad_img_dev (float32
 * [height][width] contiguous; may be NULL) and writes d/dtheta to grad_theta_dev (float64
 * triples).  (A_j, B_j) sit at their least-squares optimum, so they add no terms.
 * Enqueued. */
rd_status rd_fit_loss_backward(rd_handle h, const rd_frame* frame, const double* theta_dev,
                               const double* theta0_dev, int64_t m, double s,
                               const double* grad_loss_dev, float* grad_img_dev,
                               double* grad_theta_dev);

/* ---- the same calls over a batch of frames (one call each; the kernels are the
 * single-frame ones, enqueued frame after frame with no host synchronisation between them
 * except where a single-frame call has one).  Per-frame arrays lie back to back: ridges at
 * host offsets[i] .. offsets[i + 1] (nframes + 1 entries, offsets[0] = 0), soft
 * accumulators float32 [L][height_i][width_i] one after another, image gradients float32
 * [height_i][width_i] one after another.  widths / heights: host arrays of nframes. */

/* rd_soft_ridges over nframes frames into one list; offsets (host, nframes + 1) receive the
 * frames' starts.  RD_E_TRUNCATED if the total exceeds capacity (offsets then hold every
 * frame's count; ridges and Hessians are written up to the first frame that did not fit). */
rd_status rd_soft_ridges_batch(rd_handle h, const rd_frame* frames, int32_t nframes, const rd_params* params,
                               int32_t* xy_dev, double* hess_dev, int64_t capacity, int64_t* offsets);

/* rd_soft_forward per frame; statuses as rd_soft_forward, over the whole batch. */
rd_status rd_soft_forward_batch(rd_handle h, const int32_t* xy_dev, const double* hess_dev,
                                const int64_t* offsets, const int32_t* widths, const int32_t* heights,
                                int32_t nframes, const rd_params* params, float* acc_dev);

/* rd_soft_backward per frame; *n_isotropic (may be NULL: then enqueued) sums the frames'. */
rd_status rd_soft_backward_batch(rd_handle h, const int32_t* xy_dev, const double* hess_dev,
                                 const int64_t* offsets, const int32_t* widths, const int32_t* heights,
                                 int32_t nframes, const rd_params* params, const float* grad_acc_dev,
                                 double* grad_hess_dev, int64_t* n_isotropic);

/* rd_hessian_backward per frame, ADDING into each frame's gradient plane.  Enqueued. */
rd_status rd_hessian_backward_batch(rd_handle h, const int32_t* xy_dev, const double* grad_hess_dev,
                                    const int64_t* offsets, const int32_t* widths, const int32_t* heights,
                                    int32_t nframes, const rd_params* params, float* grad_img_dev);

/* rd_fit_loss of m rings over up to 64 device frames, ring j on frame frame_of_dev[j]
 * (int32, device; may be NULL when nframes == 1); rings with a frame index outside
 * [0, nframes) get NaN.  Enqueued. */
rd_status rd_fit_loss_batch(rd_handle h, const rd_frame* frames, int32_t nframes, const int32_t* frame_of_dev,
                            const double* theta_dev, const double* theta0_dev, int64_t m, double s,
                            double* loss_dev, double* ab_dev);

/* rd_fit_loss_backward over up to 64 frames: d/dI ADDED into the frames' gradient planes
 * (grad_img_dev may be NULL), d/dtheta per ring (NaN for rings outside the frames).
 * Enqueued. */
rd_status rd_fit_loss_backward_batch(rd_handle h, const rd_frame* frames, int32_t nframes,
                                     const int32_t* frame_of_dev, const double* theta_dev,
                                     const double* theta0_dev, int64_t m, double s,
                                     const double* grad_loss_dev, float* grad_img_dev,
                                     double* grad_theta_dev);

/* Levenberg-Marquardt refinement of m rings over up to 64 device frames (frame_of_dev[j]
 * = frame of ring j, int32; may be NULL when nframes == 1): from theta0_dev, at most
 * `iters` steps of (J^T J + lam diag J^T J) d = -J^T e on the residuals of L_j with (A, B)
 * re-solved at every point; a step is kept only if it lowers L_j (lam / 3), otherwise
 * lam x 4 (lam starts at 1e-3).  A step whose update d has every component at most tol
 * (pixels) in magnitude, kept or not, is the ring's last; a singular system gives no update
 * and does not end the loop; tol = 0 keeps the fixed count (it stops only on d = 0, which
 * every later step would repeat).  tol must be >= 0 (+inf allowed), else RD_E_INVALID.
 * Writes theta_dev and, if not NULL, loss_dev (float64) and steps_dev (int32, the steps
 * taken).  Rings with a frame index outside [0, nframes) get NaN and 0 steps.  Enqueued. */
rd_status rd_refine(rd_handle h, const rd_frame* frames, int32_t nframes,
                    const int32_t* frame_of_dev, const double* theta0_dev, int64_t m, double s,
                    int32_t iters, double tol, double* theta_dev, double* loss_dev,
                    int32_t* steps_dev);

/* ---- linking rings into trajectories, depth from radius ------------------------------
 *
 * The paper follows particles by linking each frame's rings to the previous frames' with a
 * predictive nearest-neighbour tracker that remembers missed particles for a few frames
 * (Methods, "Experimental details"), and turns a ring's radius into depth with the larger
 * root of a quadratic fit of radius against defocus (SI, calibration curve figure).  It
 * does not print the tracker; this one is (all arithmetic in float32, rounded per
 * operation, except the depth, float64 rounded to float32 once):
 *   - a track keeps its last position p = (x, y, r), a velocity v (zero until its second
 *     detection) and the frame t_l it was last seen in; ids are 0, 1, 2, ... by creation;
 *   - it takes part in frame t while t - t_l <= memory + 1, and is retired after that;
 *   - prediction p^ = p + v g with g = t - t_l; cost c = (x^-x)^2 + (y^-y)^2 + (r^-r)^2;
 *     candidates c <= gate^2;
 *   - greedy matching: candidates in increasing (c, track id, detection index) order, each
 *     taken when both of its ends are still free;
 *   - a matched track gets v = (d - p) / g, p = d, t_l = t; each unmatched detection opens a
 *     track (v = 0), ids in increasing detection order;
 *   - depth z(r) = larger root of c2 z^2 + c1 z + c0 - r = 0 for c2 > 0, the discriminant
 *     clamped at 0.
 * The paper's linker also accounts for accelerations in its kinematic model (Methods,
 * "Precision assessment").  With model = RD_LINK_ACCELERATION a track keeps its last three
 * detections (t_k, q_k), t_0 < t_1 < t_2 = t_l (fewer while it is young), and predicts with
 * the polynomial through them at frame t in Lagrange form: p^ = q_2 with one detection,
 * w_2 q_2 + w_1 q_1 with two, (w_2 q_2 + w_1 q_1) + w_0 q_0 with three, where
 * w_k = prod_{m != k} (t - t_m) / prod_{m != k} (t_k - t_m), numerator and denominator exact
 * integers converted to float32 and divided in float32; a match appends (t, d) and drops
 * the oldest detection beyond three.  Gate, memory, matching and ids are as above. */

#define RD_LINK_VELOCITY 0             /* prediction p + v g                         */
#define RD_LINK_ACCELERATION 1         /* polynomial through the last three detections */
#define RD_LINK_MAX_DETECTIONS 4096   /* detections in one frame                    */
#define RD_LINK_MAX_ACTIVE 6144       /* tracks taking part in one frame            */

typedef struct {
    float gate;        /* > 0: largest distance in (x, y, r) space of a link, px        */
    int32_t memory;    /* >= 0: frames a track may miss and still be continued          */
    double depth_c0;   /* radius calibration r(z) = c0 + c1 z + c2 z^2; all finite and
                          c2 > 0, else rd_linker_create returns RD_E_INVALID              */
    double depth_c1;
    double depth_c2;
    int32_t model;     /* RD_LINK_VELOCITY or RD_LINK_ACCELERATION                      */
} rd_link_params;

typedef struct rd_linker_s* rd_linker;

/* A linker: device state for up to max_tracks tracks over the whole sequence and calls of
 * up to max_frames frames.  Work is ordered on `stream` (hipStream_t; NULL = default) on the
 * current device.  RD_E_INVALID for bad parameters, RD_E_NOMEM if allocation fails. */
rd_status rd_linker_create(const rd_link_params* params, int32_t max_tracks, int32_t max_frames,
                           void* stream, rd_linker* out);
void rd_linker_destroy(rd_linker linker);

/* Forget every track; the next frame is frame 0 again. */
rd_status rd_linker_reset(rd_linker linker);

/* Tracks opened so far, tracks taking part in the next frame, frames linked so far.
 * RD_E_OVERFLOW if a capacity was exceeded since the last reset (the state is then
 * invalid until rd_linker_reset). */
rd_status rd_linker_info(rd_linker linker, int32_t* ntracks, int32_t* nactive, int32_t* frame);

/* Link the next nframes frames (1 <= nframes <= max_frames).  det_dev: float32 (x, y, r)
 * triples, device, frames back to back; frame_offsets: host, nframes + 1 prefix offsets
 * into det_dev in detections, starting at 0, each frame <= RD_LINK_MAX_DETECTIONS
 * (RD_E_TOO_LARGE otherwise).  Writes ids_dev[k] (int32, device) = the track id of
 * detection k, and, if z_dev (float32, device) is not NULL, its depth.  Completed on
 * return.  RD_E_OVERFLOW if more than max_tracks tracks, RD_LINK_MAX_ACTIVE tracks taking
 * part in a frame, or 2^20 candidate pairs in a frame were needed.  In the frame where that
 * happens, the detections that could not open a track get id -1 (the others are linked, or
 * open the tracks that still fit, in detection order); every later frame, in this call and
 * the following ones, gets id -1 for all of its detections (depths are still written) until
 * rd_linker_reset.  rd_linker_info then reports at most max_tracks tracks. */
rd_status rd_link(rd_linker linker, const float* det_dev, const int32_t* frame_offsets,
                  int32_t nframes, int32_t* ids_dev, float* z_dev);

#ifdef __cplusplus
}
#endif

#endif /* RIDGE_DETECT_H */
