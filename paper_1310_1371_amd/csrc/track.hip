// Frame-to-frame linking of detected rings into trajectories, and depth from radius.
//
// The paper links its per-frame ring lists with a predictive nearest-neighbour tracker that
// has a memory for missed frames (Methods, "Experimental details"), and converts a ring's
// radius into depth through the larger root of a quadratic calibration (SI, calibration
// curve figure).  The tracker itself is not printed; the one here:
//   prediction p^ = p + v g (g = frames since the track was last seen), or, in the
//   acceleration model (the paper's linker accounts for accelerations: Methods, "Precision
//   assessment"), the Lagrange polynomial through the track's last three detections at
//   their frames; cost c = |p^ - d|^2 over (x, y, r), candidates c <= gate^2, and the greedy
//   matching that takes candidates in increasing (c, track id, detection index) order.
//
// The greedy matching is found without sorting: with a strict total order on the candidate
// pairs, the greedy result is the union of rounds of "locally dominant" pairs, each pair the
// smallest at both of its ends among the pairs still free (a classical property of greedy
// matching).  Every round is two passes of LDS atomicMin over the candidate list, with
// 64-bit keys (cost bits << 32 | other end) that order exactly as (c, i, j).  The cost is
// float32, and non-negative, so its bit pattern orders like its value.
//
// One workgroup walks the frames in order (each frame depends on the previous one).  The
// frame's detections sit in LDS, counting-sorted into a hashed grid of cells at least
// 1.125 gate wide; each thread looks up its tracks' candidates in the 3 x 3 cells around the
// prediction.  Track state lives in device memory between calls.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "ridge_detect.h"

#define RD_LINK_HIP(call)                              \
    do {                                               \
        if ((call) != hipSuccess) return RD_E_DEVICE;  \
    } while (0)

namespace rd_track {

constexpr int THREADS = 1024;
constexpr int MAX_DET = RD_LINK_MAX_DETECTIONS;   // detections of one frame
constexpr int MAX_ACTIVE = RD_LINK_MAX_ACTIVE;    // tracks taking part in one frame
constexpr uint64_t FREE = ~0ull;

enum { S_NTRACKS = 0, S_NACTIVE, S_FRAME, S_CUR, S_ERR, S_COUNT };
enum { ERR_ACTIVE = 1, ERR_TRACKS = 2, ERR_EDGES = 4 };

struct Args {
    const float* det;          // 3 floats (x, y, r) per detection, frames back to back
    const int32_t* offsets;    // nframes + 1 prefix offsets into det
    int32_t nframes;
    int32_t* ids;              // out: track id per detection (-1 after an overflow)
    float* z;                  // out: depth per detection, or null
    double c0, c1, c2;
    float gate;
    int32_t memory;
    int32_t model;             // RD_LINK_VELOCITY or RD_LINK_ACCELERATION
    float* pos;                // 3 floats per track: last (x, y, r)
    float* vel;                // 3 floats per track (velocity model)
    int32_t* t_last;           // per track
    float* hist;               // acceleration model: 6 floats per track, q_0 then q_1
    int32_t* hist_t;           // acceleration model: 2 ints per track, t_0 then t_1 (-1: none)
    int32_t* act0;             // active lists, double-buffered across frames
    int32_t* act1;
    int32_t* state;            // S_COUNT words
    int32_t max_tracks;
    uint4* edges;              // candidate pairs of one frame: (cost bits, slot, det, id)
    int32_t max_edges;
};

__device__ inline uint64_t key(uint32_t cbits, uint32_t other) { return (uint64_t(cbits) << 32) | other; }

// Candidate search grid: square cells of side cs >= 1.125 gate hashed into NB buckets.  A
// pair within the gate is at most gate (1 + 1e-6) apart along x and along y, under 0.89 cs,
// so its cells differ by at most one even after the products v / cs are rounded (each off
// by at most 2^-6 cells while |v| < 2^17 and cs >= 1/4).  Coordinates beyond that, and
// non-finite ones, take the exhaustive scan instead, so the candidate set is always exactly
// the pairs that pass the cost test.
constexpr int NB = 4096;
constexpr float NEAR = 131072.f;
__device__ inline bool near(float v) { return fabsf(v) < NEAR; }
__device__ inline int cell(float v, float inv_cs) { return (int)floorf(v * inv_cs); }
__device__ inline int bucket(int cx, int cy) {
    uint32_t h = (uint32_t)cx * 0x9E3779B1u ^ (uint32_t)cy * 0x85EBCA77u;
    return (int)((h ^ (h >> 15)) & (NB - 1));
}

__global__ __launch_bounds__(THREADS) void k_link(Args A) {
#pragma clang fp contract(off)
    __shared__ float sx[MAX_DET], sy[MAX_DET], sr[MAX_DET];   // detections
    __shared__ unsigned long long bt[MAX_ACTIVE];       // best key per active slot
    __shared__ unsigned long long bd[MAX_DET];          // best key per detection
    __shared__ int16_t md[MAX_DET];                     // matched slot + 1, 0 = free
    __shared__ uint8_t mt[MAX_ACTIVE];                  // slot matched
    __shared__ int32_t s_ne, s_keep, s_changed, s_err, s_wave[THREADS / 64], s_base, s_far;
    // The grid lives in bd's storage and its prefix scan in bt's: both are initialised only
    // after the candidate search.  A detection's rank within its bucket waits in md.
    uint32_t* gstart = reinterpret_cast<uint32_t*>(bd);                  // NB bucket starts
    uint16_t* gidx = reinterpret_cast<uint16_t*>(gstart + NB);           // detections by bucket
    int32_t* stmp = reinterpret_cast<int32_t*>(bt);                      // THREADS partial sums
    static_assert(NB * 4 + MAX_DET * 2 <= MAX_DET * 8, "grid must fit in bd");
    static_assert(THREADS * 4 <= MAX_ACTIVE * 8 && NB == 4 * THREADS, "scan layout");

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int ntracks = A.state[S_NTRACKS], nact = A.state[S_NACTIVE], t = A.state[S_FRAME];
    int cur = A.state[S_CUR];
    if (tid == 0) s_err = A.state[S_ERR];
    const float g2 = A.gate * A.gate;
    const float inv_cs = 1.0f / fmaxf(1.125f * A.gate, 0.25f);
    auto depth = [&](float r) {
        double disc = A.c1 * A.c1 - 4.0 * A.c2 * (A.c0 - (double)r);
        disc = disc < 0.0 ? 0.0 : disc;          // a NaN radius stays NaN
        return (float)((-A.c1 + sqrt(disc)) / (2.0 * A.c2));
    };
    __syncthreads();

    for (int f = 0; f < A.nframes; ++f) {
        const int d0 = A.offsets[f], n = A.offsets[f + 1] - d0;   // n <= MAX_DET, checked on the host
        // After an overflow the track state is incomplete: no frame is linked until a reset,
        // every id is -1 (s_err is read by all threads between the barriers that end a frame
        // and the first barrier of this one, and written only after that barrier).
        if (s_err != 0) {
            for (int j = tid; j < n; j += THREADS) {
                A.ids[d0 + j] = -1;
                if (A.z) A.z[d0 + j] = depth(A.det[3 * (int64_t)(d0 + j) + 2]);
            }
            t += 1;
            continue;
        }
        const int32_t* act_in = cur ? A.act1 : A.act0;
        int32_t* act_out = cur ? A.act0 : A.act1;
        for (int j = tid; j < n; j += THREADS) {
            const float* p = A.det + 3 * (int64_t)(d0 + j);
            sx[j] = p[0];
            sy[j] = p[1];
            sr[j] = p[2];
        }
        for (int b = tid; b < NB; b += THREADS) gstart[b] = 0;
        if (tid == 0) { s_ne = 0; s_keep = 0; s_changed = 0; s_far = 0; }
        __syncthreads();

        // Counting sort of the detections into the grid's buckets.
        for (int j = tid; j < n; j += THREADS) {
            const float x = sx[j], y = sy[j];
            if (near(x) && near(y)) md[j] = (int16_t)atomicAdd(&gstart[bucket(cell(x, inv_cs), cell(y, inv_cs))], 1u);
            else { md[j] = -1; s_far = 1; }
        }
        __syncthreads();
        uint32_t c4[4], run = 0;
        for (int k = 0; k < 4; ++k) { c4[k] = gstart[4 * tid + k]; run += c4[k]; }
        stmp[tid] = (int32_t)run;
        __syncthreads();
        for (int off = 1; off < THREADS; off <<= 1) {
            const int32_t v = tid >= off ? stmp[tid - off] : 0;
            __syncthreads();
            stmp[tid] += v;
            __syncthreads();
        }
        const int total = stmp[THREADS - 1];
        run = (uint32_t)stmp[tid] - run;
        for (int k = 0; k < 4; ++k) { gstart[4 * tid + k] = run; run += c4[k]; }
        __syncthreads();
        for (int j = tid; j < n; j += THREADS)
            if (md[j] >= 0) gidx[gstart[bucket(cell(sx[j], inv_cs), cell(sy[j], inv_cs))] + md[j]] = (uint16_t)j;
        __syncthreads();
        const bool far_frame = s_far != 0;

        // Tracks still taking part keep a slot in the next active list and emit candidates.
        for (int a = tid; a < nact; a += THREADS) {
            const int i = act_in[a];
            const int gap = t - A.t_last[i];
            if (gap > A.memory + 1) continue;               // retired
            const int slot = atomicAdd(&s_keep, 1);
            if (slot >= MAX_ACTIVE) { atomicOr(&s_err, ERR_ACTIVE); continue; }
            act_out[slot] = i;
            float px, py, pr;
            if (A.model == RD_LINK_VELOCITY) {
                const float g = (float)gap;
                px = A.pos[3 * i] + A.vel[3 * i] * g;
                py = A.pos[3 * i + 1] + A.vel[3 * i + 1] * g;
                pr = A.pos[3 * i + 2] + A.vel[3 * i + 2] * g;
            } else {
                const int64_t t2 = A.t_last[i], t1 = A.hist_t[2 * i + 1], t0 = A.hist_t[2 * i];
                const float* q1 = A.hist + 6 * (int64_t)i + 3;
                const float* q0 = A.hist + 6 * (int64_t)i;
                px = A.pos[3 * i];
                py = A.pos[3 * i + 1];
                pr = A.pos[3 * i + 2];
                if (t1 >= 0 && t0 < 0) {                      // the line through two
                    const float w2 = (float)(t - t1) / (float)(t2 - t1);
                    const float w1 = (float)(t - t2) / (float)(t1 - t2);
                    px = w2 * px + w1 * q1[0];
                    py = w2 * py + w1 * q1[1];
                    pr = w2 * pr + w1 * q1[2];
                } else if (t1 >= 0) {                         // the parabola through three
                    const float w2 = (float)((t - t1) * (t - t0)) / (float)((t2 - t1) * (t2 - t0));
                    const float w1 = (float)((t - t2) * (t - t0)) / (float)((t1 - t2) * (t1 - t0));
                    const float w0 = (float)((t - t2) * (t - t1)) / (float)((t0 - t2) * (t0 - t1));
                    px = (w2 * px + w1 * q1[0]) + w0 * q0[0];
                    py = (w2 * py + w1 * q1[1]) + w0 * q0[1];
                    pr = (w2 * pr + w1 * q1[2]) + w0 * q0[2];
                }
            }
            auto test = [&](int j) {
                const float dx = px - sx[j], dy = py - sy[j], dr = pr - sr[j];
                const float c = dx * dx + dy * dy + dr * dr;
                if (c <= g2) {
                    const int e = atomicAdd(&s_ne, 1);
                    if (e < A.max_edges) A.edges[e] = make_uint4(__float_as_uint(c), slot, j, i);
                    else atomicOr(&s_err, ERR_EDGES);
                }
            };
            if (far_frame || !near(px) || !near(py)) {
                for (int j = 0; j < n; ++j) test(j);
            } else {
                const int cx = cell(px, inv_cs), cy = cell(py, inv_cs);
                int bs[9];
#pragma unroll
                for (int k = 0; k < 9; ++k) bs[k] = bucket(cx + k % 3 - 1, cy + k / 3 - 1);
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    bool dup = false;          // two cells hashed to one bucket: scan it once
#pragma unroll
                    for (int m = 0; m < k; ++m) dup |= bs[m] == bs[k];
                    if (dup) continue;
                    const int end = bs[k] + 1 < NB ? (int)gstart[bs[k] + 1] : total;
                    for (int q = (int)gstart[bs[k]]; q < end; ++q) test(gidx[q]);
                }
            }
        }
        __syncthreads();
        const int keep = min(s_keep, MAX_ACTIVE);
        const int ne = min(s_ne, A.max_edges);
        for (int a = tid; a < keep; a += THREADS) { bt[a] = FREE; mt[a] = 0; }
        for (int j = tid; j < n; j += THREADS) { bd[j] = FREE; md[j] = 0; }

        // Rounds of locally dominant pairs.  Every round with a free candidate matches at
        // least the smallest free one, so the loop ends after at most ne + 1 rounds.
        for (;;) {
            __syncthreads();
            for (int e = tid; e < ne; e += THREADS) {
                const uint4 E = A.edges[e];
                if (mt[E.y] || md[E.z]) continue;
                atomicMin(&bt[E.y], key(E.x, E.z));
                atomicMin(&bd[E.z], key(E.x, E.w));
            }
            __syncthreads();
            for (int e = tid; e < ne; e += THREADS) {
                const uint4 E = A.edges[e];
                if (mt[E.y] || md[E.z]) continue;
                if (bt[E.y] == key(E.x, E.z) && bd[E.z] == key(E.x, E.w)) {
                    mt[E.y] = 1;
                    md[E.z] = (int16_t)(E.y + 1);
                    s_changed = 1;
                }
            }
            __syncthreads();
            const int changed = s_changed;
            __syncthreads();
            if (!changed) break;
            for (int a = tid; a < keep; a += THREADS)
                if (!mt[a]) bt[a] = FREE;
            for (int j = tid; j < n; j += THREADS)
                if (!md[j]) bd[j] = FREE;
            if (tid == 0) s_changed = 0;
        }

        // Matched tracks move; unmatched detections open tracks, ids by detection index.
        if (tid == 0) s_base = 0;
        __syncthreads();
        for (int j0 = 0; j0 < n; j0 += THREADS) {
            const int j = j0 + tid;
            const bool fresh = j < n && md[j] == 0;
            const uint64_t bal = __ballot(fresh);
            if (lane == 0) s_wave[wave] = __popcll(bal);
            __syncthreads();
            int before = s_base;
            for (int w = 0; w < wave; ++w) before += s_wave[w];
            before += __popcll(bal & ((1ull << lane) - 1));
            if (j < n) {
                const float4 d = make_float4(sx[j], sy[j], sr[j], 0.f);
                int id;
                if (!fresh) {
                    id = act_out[(int)md[j] - 1];
                    if (A.model == RD_LINK_VELOCITY) {
                        const float g = (float)(t - A.t_last[id]);
                        A.vel[3 * id] = (d.x - A.pos[3 * id]) / g;
                        A.vel[3 * id + 1] = (d.y - A.pos[3 * id + 1]) / g;
                        A.vel[3 * id + 2] = (d.z - A.pos[3 * id + 2]) / g;
                    } else {                                  // the history moves down one
                        float* h = A.hist + 6 * (int64_t)id;
                        for (int c = 0; c < 3; ++c) {
                            h[c] = h[3 + c];
                            h[3 + c] = A.pos[3 * id + c];
                        }
                        A.hist_t[2 * id] = A.hist_t[2 * id + 1];
                        A.hist_t[2 * id + 1] = A.t_last[id];
                    }
                } else {
                    id = ntracks + before;
                    const int slot = keep + before;
                    if (id >= A.max_tracks) { atomicOr(&s_err, ERR_TRACKS); id = -1; }
                    else if (slot >= MAX_ACTIVE) { atomicOr(&s_err, ERR_ACTIVE); id = -1; }
                    else {
                        act_out[slot] = id;
                        if (A.model == RD_LINK_VELOCITY) {
                            A.vel[3 * id] = 0.f;
                            A.vel[3 * id + 1] = 0.f;
                            A.vel[3 * id + 2] = 0.f;
                        } else {
                            A.hist_t[2 * id] = -1;
                            A.hist_t[2 * id + 1] = -1;
                        }
                    }
                }
                if (id >= 0) {
                    A.pos[3 * id] = d.x;
                    A.pos[3 * id + 1] = d.y;
                    A.pos[3 * id + 2] = d.z;
                    A.t_last[id] = t;
                }
                A.ids[d0 + j] = id;
                if (A.z) A.z[d0 + j] = depth(d.z);
            }
            __syncthreads();
            if (tid == 0) for (int w = 0; w < THREADS / 64; ++w) s_base += s_wave[w];
            __syncthreads();   // s_wave is rewritten by the next step
        }
        __syncthreads();
        // Fresh detections take ids ntracks + rank and slots keep + rank in detection order, so
        // the ones that got both are exactly the first min(nnew, max_tracks - ntracks,
        // MAX_ACTIVE - keep); only those become tracks and active slots.
        const int made = min(s_base, min(A.max_tracks - ntracks, MAX_ACTIVE - keep));
        ntracks += made;
        nact = keep + made;
        t += 1;
        cur ^= 1;
        __syncthreads();   // act_out, positions and LDS reuse ordered before the next frame
    }
    if (tid == 0) {
        A.state[S_NTRACKS] = ntracks;
        A.state[S_NACTIVE] = nact;
        A.state[S_FRAME] = t;
        A.state[S_CUR] = cur;
        A.state[S_ERR] = s_err;
    }
}

}  // namespace rd_track

using namespace rd_track;

struct rd_linker_s {
    rd_link_params p{};
    int32_t max_tracks = 0, max_edges = 0;
    hipStream_t stream = nullptr;
    float *pos = nullptr, *vel = nullptr, *hist = nullptr;
    int32_t *t_last = nullptr, *hist_t = nullptr, *act0 = nullptr, *act1 = nullptr, *state = nullptr, *offsets = nullptr;
    uint4* edges = nullptr;
    int32_t max_frames = 0;
    int32_t* h_state = nullptr;   // pinned
};

static void linker_free(rd_linker_s* L) {
    (void)hipFree(L->pos); (void)hipFree(L->vel); (void)hipFree(L->t_last); (void)hipFree(L->act0); (void)hipFree(L->act1);
    (void)hipFree(L->hist); (void)hipFree(L->hist_t);
    (void)hipFree(L->state); (void)hipFree(L->offsets); (void)hipFree(L->edges);
    if (L->h_state) (void)hipHostFree(L->h_state);
    delete L;
}

static bool link_params_ok(const rd_link_params* p) {
    return p && p->gate > 0.f && p->gate < 1e18f && p->memory >= 0 && p->memory < (1 << 20) &&
           std::isfinite(p->depth_c0) && std::isfinite(p->depth_c1) && std::isfinite(p->depth_c2) &&
           p->depth_c2 > 0.0 && (p->model == RD_LINK_VELOCITY || p->model == RD_LINK_ACCELERATION);
}

extern "C" rd_status rd_linker_create(const rd_link_params* params, int32_t max_tracks,
                                      int32_t max_frames, void* stream, rd_linker* out) {
    if (!out || !link_params_ok(params) || max_tracks < 1 || max_tracks > (1 << 28) || max_frames < 1 ||
        max_frames > (1 << 20))
        return RD_E_INVALID;
    *out = nullptr;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return RD_E_DEVICE;
    auto* L = new rd_linker_s;
    L->p = *params;
    L->max_tracks = max_tracks;
    L->max_frames = max_frames;
    L->max_edges = 1 << 20;
    L->stream = (hipStream_t)stream;
    const size_t nt = (size_t)max_tracks;
    if (hipMalloc(&L->pos, nt * 3 * sizeof(float)) != hipSuccess ||
        hipMalloc(&L->vel, nt * 3 * sizeof(float)) != hipSuccess ||
        hipMalloc(&L->t_last, nt * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&L->act0, MAX_ACTIVE * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&L->act1, MAX_ACTIVE * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&L->state, S_COUNT * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&L->offsets, ((size_t)max_frames + 1) * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&L->edges, (size_t)L->max_edges * sizeof(uint4)) != hipSuccess ||
        hipHostMalloc(&L->h_state, S_COUNT * sizeof(int32_t)) != hipSuccess ||
        (params->model == RD_LINK_ACCELERATION &&
         (hipMalloc(&L->hist, nt * 6 * sizeof(float)) != hipSuccess ||
          hipMalloc(&L->hist_t, nt * 2 * sizeof(int32_t)) != hipSuccess))) {
        linker_free(L);
        return RD_E_NOMEM;
    }
    if (hipMemsetAsync(L->state, 0, S_COUNT * sizeof(int32_t), L->stream) != hipSuccess ||
        hipStreamSynchronize(L->stream) != hipSuccess) {
        linker_free(L);
        return RD_E_DEVICE;
    }
    *out = L;
    return RD_OK;
}

extern "C" void rd_linker_destroy(rd_linker L) {
    if (!L) return;
    (void)hipStreamSynchronize(L->stream);
    linker_free(L);
}

extern "C" rd_status rd_linker_reset(rd_linker L) {
    if (!L) return RD_E_INVALID;
    RD_LINK_HIP(hipMemsetAsync(L->state, 0, S_COUNT * sizeof(int32_t), L->stream));
    RD_LINK_HIP(hipStreamSynchronize(L->stream));
    return RD_OK;
}

extern "C" rd_status rd_linker_info(rd_linker L, int32_t* ntracks, int32_t* nactive, int32_t* frame) {
    if (!L) return RD_E_INVALID;
    RD_LINK_HIP(hipMemcpyAsync(L->h_state, L->state, S_COUNT * sizeof(int32_t), hipMemcpyDeviceToHost, L->stream));
    RD_LINK_HIP(hipStreamSynchronize(L->stream));
    if (ntracks) *ntracks = L->h_state[S_NTRACKS];
    if (nactive) *nactive = L->h_state[S_NACTIVE];
    if (frame) *frame = L->h_state[S_FRAME];
    return L->h_state[S_ERR] ? RD_E_OVERFLOW : RD_OK;
}

extern "C" rd_status rd_link(rd_linker L, const float* det_dev, const int32_t* frame_offsets,
                             int32_t nframes, int32_t* ids_dev, float* z_dev) {
    if (!L || !frame_offsets || nframes < 1 || nframes > L->max_frames) return RD_E_INVALID;
    if (frame_offsets[0] != 0) return RD_E_INVALID;
    for (int f = 0; f < nframes; ++f) {
        const int64_t n = (int64_t)frame_offsets[f + 1] - frame_offsets[f];
        if (n < 0) return RD_E_INVALID;
        if (n > MAX_DET) return RD_E_TOO_LARGE;
    }
    if (frame_offsets[nframes] > 0 && (!det_dev || !ids_dev)) return RD_E_INVALID;
    RD_LINK_HIP(hipMemcpyAsync(L->offsets, frame_offsets, ((size_t)nframes + 1) * sizeof(int32_t),
                               hipMemcpyHostToDevice, L->stream));
    Args a{};
    a.det = det_dev;
    a.offsets = L->offsets;
    a.nframes = nframes;
    a.ids = ids_dev;
    a.z = z_dev;
    a.c0 = L->p.depth_c0;
    a.c1 = L->p.depth_c1;
    a.c2 = L->p.depth_c2;
    a.gate = L->p.gate;
    a.memory = L->p.memory;
    a.model = L->p.model;
    a.pos = L->pos;
    a.vel = L->vel;
    a.t_last = L->t_last;
    a.hist = L->hist;
    a.hist_t = L->hist_t;
    a.act0 = L->act0;
    a.act1 = L->act1;
    a.state = L->state;
    a.max_tracks = L->max_tracks;
    a.edges = L->edges;
    a.max_edges = L->max_edges;
    hipLaunchKernelGGL(k_link, dim3(1), dim3(THREADS), 0, L->stream, a);
    RD_LINK_HIP(hipGetLastError());
    return rd_linker_info(L, nullptr, nullptr, nullptr);
}
