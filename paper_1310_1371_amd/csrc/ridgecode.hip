// Encoded ridge streams: the ridges of a frame (pixel and direction code) in a compact form
// that can stand in for the frame after step 2 (SI, "Additional notes": ridge coordinates
// with their directions as a compressed representation of the image).
//
// Stream of one frame (little endian, 16-byte aligned):
//   [0, 16)        u32 magic "RDR1", u16 width, u16 height, u32 ridge count n, u32 zero
//   [16, ...)      u16 ridge count of every 16x16 pixel bin, bins in raster order
//   then           u8 per ridge: its pixel within its bin, (y & 15) << 4 | (x & 15), the
//                  ridges bin after bin
//   then           zero padding to a multiple of 4 bytes
//   then           u32 per ridge, in the same order: qx (low 16 bits) | qy << 16
//   then           zero padding to a multiple of 16 bytes
// About 5 bytes per ridge plus 2 per 256 pixels.
//
// Both directions work on chunks of 256 bins.  A first kernel (one workgroup per frame)
// turns the bin counts into the record index of every chunk's first ridge; encoding then
// places each frame's stream after the previous frames' (one small kernel), and a
// workgroup per chunk moves its ridges between the context's bins and the stream.
#include "rd_internal.h"

namespace rd {
namespace {

constexpr int SNT = 1024;    // threads of the per-frame scan
constexpr int CNT = RIDGE_CHUNK;

__device__ __forceinline__ uint32_t incl_scan64(uint32_t v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t n = __shfl_up(v, o, 64);
        if (lane >= o) v += n;
    }
    return v;
}

// count of bin b of frame f: from the context's bins (encode) or the stream (decode)
template <bool ENC>
__device__ __forceinline__ uint32_t bin_count_of(const RidgeCodeArgs& a, const FrameDesc& fd, int f, int64_t b,
                                                 bool* bad) {
    if (ENC) return min(a.bin_count[fd.bin0 + b], static_cast<uint32_t>(BIN_CAP));
    const uint16_t c = reinterpret_cast<const uint16_t*>(a.enc + a.offsets[f] + 16)[b];
    if (c > BIN_CAP) *bad = true;
    return min(static_cast<uint32_t>(c), static_cast<uint32_t>(BIN_CAP));
}

// One workgroup per frame: each thread sums a contiguous run of bins, the runs are scanned
// across the workgroup, and every chunk start in a run gets its record base.
template <bool ENC>
__global__ __launch_bounds__(SNT) void k_chunk_scan(RidgeCodeArgs a) {
    __shared__ uint32_t sWave[SNT / 64];
    const int f = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const FrameDesc fd = a.frames[f];
    const int64_t nbins = static_cast<int64_t>(fd.nbx) * fd.nby;
    const int64_t seg = (nbins + SNT - 1) / SNT;
    const int64_t b0 = min(nbins, seg * tid), b1 = min(nbins, b0 + seg);
    bool bad = false;
    uint32_t sum = 0;
    for (int64_t b = b0; b < b1; ++b) sum += bin_count_of<ENC>(a, fd, f, b, &bad);
    const uint32_t inc = incl_scan64(sum, lane);
    if (lane == 63) sWave[wave] = inc;
    __syncthreads();
    uint32_t run = inc - sum, total = 0;
#pragma unroll
    for (int w = 0; w < SNT / 64; ++w) {
        if (w < wave) run += sWave[w];
        total += sWave[w];
    }
    const uint32_t c0 = a.chunk0[f];
    for (int64_t b = b0; b < b1; ++b) {
        if ((b & (CNT - 1)) == 0) a.cbase[c0 + b / CNT] = run;
        run += bin_count_of<ENC>(a, fd, f, b, &bad);
    }
    if (tid == 0) {
        a.frame_n[f] = total;
        if (!ENC) {
            const uint32_t n_hdr = reinterpret_cast<const uint32_t*>(a.enc + a.offsets[f])[2];
            if (n_hdr != total) atomicOr(a.flags, 1u);
        }
    }
    if (bad) atomicOr(a.flags, 1u);
}

// Encode: the streams one after another, each 16-byte aligned.
__global__ void k_stream_offsets(RidgeCodeArgs a) {
    if (threadIdx.x != 0) return;
    int64_t off = 0;
    for (int f = 0; f < a.nframes; ++f) {
        a.offsets[f] = off;
        const FrameDesc fd = a.frames[f];
        off += ridge_stream_bytes(a.frame_n[f], static_cast<int64_t>(fd.nbx) * fd.nby);
    }
    a.offsets[a.nframes] = off;
}

// the frame a chunk belongs to (chunk0 is ascending)
__device__ __forceinline__ int frame_of_chunk(const RidgeCodeArgs& a, uint32_t c) {
    int lo = 0, hi = a.nframes;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (a.chunk0[mid] <= c) lo = mid; else hi = mid;
    }
    return lo;
}

// Exclusive scan of one count per thread over the workgroup into sPre[0 .. CNT].
__device__ __forceinline__ void chunk_scan(uint32_t cnt, uint32_t* sPre, uint32_t* sWave) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t inc = incl_scan64(cnt, lane);
    if (lane == 63) sWave[wave] = inc;
    __syncthreads();
    uint32_t base = 0, total = 0;
#pragma unroll
    for (int w = 0; w < CNT / 64; ++w) {
        if (w < wave) base += sWave[w];
        total += sWave[w];
    }
    sPre[tid] = base + inc - cnt;
    if (tid == 0) sPre[CNT] = total;
    __syncthreads();
}

// largest t with sPre[t] <= k
__device__ __forceinline__ int find_bin(const uint32_t* sPre, uint32_t k) {
    int lo = 0, hi = CNT;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (sPre[mid] <= k) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(CNT) void k_encode_chunk(RidgeCodeArgs a) {
    __shared__ uint32_t sPre[CNT + 1];
    __shared__ uint32_t sWave[CNT / 64];
    const uint32_t cg = blockIdx.x;
    const int f = frame_of_chunk(a, cg), tid = threadIdx.x;
    const FrameDesc fd = a.frames[f];
    const int64_t nbins = static_cast<int64_t>(fd.nbx) * fd.nby;
    const int64_t c = cg - a.chunk0[f];
    const int64_t b0 = c * CNT;
    const int64_t n = a.frame_n[f];
    const int64_t off = a.offsets[f];
    if (off + ridge_stream_bytes(n, nbins) > a.capacity) return;     // reported as truncated
    uint8_t* const st = a.enc + off;
    const int64_t qoff = ridge_stream_qoff(n, nbins);
    const int64_t b = b0 + tid;
    uint32_t cnt = 0;
    if (b < nbins) {
        cnt = min(a.bin_count[fd.bin0 + b], static_cast<uint32_t>(BIN_CAP));
        reinterpret_cast<uint16_t*>(st + 16)[b] = static_cast<uint16_t>(cnt);
    }
    chunk_scan(cnt, sPre, sWave);
    const uint32_t base = a.cbase[cg];
    for (uint32_t k = tid; k < sPre[CNT]; k += CNT) {
        const int t = find_bin(sPre, k);
        const int64_t slot = (fd.bin0 + b0 + t) * BIN_CAP + (k - sPre[t]);
        const uint32_t xy = a.rxy[slot];
        st[16 + 2 * nbins + base + k] = static_cast<uint8_t>((((xy >> 16) & 15u) << 4) | (xy & 15u));
        reinterpret_cast<uint32_t*>(st + qoff)[base + k] = a.rq[slot];
    }
    if (c == 0 && tid == 0) {
        uint32_t* const h = reinterpret_cast<uint32_t*>(st);
        h[0] = RIDGE_MAGIC;
        h[1] = static_cast<uint32_t>(fd.W) | (static_cast<uint32_t>(fd.H) << 16);
        h[2] = static_cast<uint32_t>(n);
        h[3] = 0u;
        for (int64_t i = 16 + 2 * nbins + n; i < qoff; ++i) st[i] = 0;
        for (int64_t i = qoff + 4 * n; i < ridge_stream_bytes(n, nbins); ++i) st[i] = 0;
    }
}

// Decode one chunk into the context's bins, checking each ridge: inside the frame, a
// direction code step 1 can make, its pixel not listed before (one bit per pixel).
__global__ __launch_bounds__(CNT) void k_decode_chunk(RidgeCodeArgs a) {
    __shared__ uint32_t sPre[CNT + 1];
    __shared__ uint32_t sWave[CNT / 64];
    __shared__ uint32_t sMask[CNT * 8];
    const uint32_t cg = blockIdx.x;
    const int f = frame_of_chunk(a, cg), tid = threadIdx.x;
    const FrameDesc fd = a.frames[f];
    const int64_t nbins = static_cast<int64_t>(fd.nbx) * fd.nby;
    const int64_t c = cg - a.chunk0[f];
    const int64_t b0 = c * CNT;
    const uint8_t* const st = a.enc + a.offsets[f];
    const int64_t n = reinterpret_cast<const uint32_t*>(st)[2];          // the header's count
    const int64_t qoff = ridge_stream_qoff(n, nbins);
    for (int i = tid; i < CNT * 8; i += CNT) sMask[i] = 0u;
    const int64_t b = b0 + tid;
    uint32_t cnt = 0;
    if (b < nbins) {
        cnt = min(static_cast<uint32_t>(reinterpret_cast<const uint16_t*>(st + 16)[b]), static_cast<uint32_t>(BIN_CAP));
        a.bin_count[fd.bin0 + b] = cnt;
    }
    chunk_scan(cnt, sPre, sWave);
    const uint32_t base = a.cbase[cg];
    uint32_t bad = 0;
    for (uint32_t k = tid; k < sPre[CNT]; k += CNT) {
        if (base + k >= n) {                 // the counts claim more ridges than the header
            bad |= 1u;
            break;
        }
        const int t = find_bin(sPre, k);
        const int64_t bin = b0 + t;
        const uint32_t pos = st[16 + 2 * nbins + base + k];
        const uint32_t q = reinterpret_cast<const uint32_t*>(st + qoff)[base + k];
        const int x = static_cast<int>((bin % fd.nbx) * BIN + (pos & 15u));
        const int y = static_cast<int>((bin / fd.nbx) * BIN + (pos >> 4));
        if (x >= fd.W || y >= fd.H) bad |= 2u;
        if (!ridge_code_ok(static_cast<int16_t>(q & 0xffffu), static_cast<int16_t>(q >> 16))) bad |= 4u;
        const uint32_t bit = 1u << (pos & 31u);
        if (atomicOr(&sMask[t * 8 + (pos >> 5)], bit) & bit) bad |= 8u;
        const int64_t slot = (fd.bin0 + bin) * BIN_CAP + (k - sPre[t]);
        a.rxy[slot] = static_cast<uint32_t>(x) | (static_cast<uint32_t>(y) << 16);
        a.rq[slot] = q;
        a.rk[slot] = 0.0f;
    }
    if (bad) atomicOr(a.flags, bad);
}

}  // namespace

hipError_t launch_ridge_encode(const RidgeCodeArgs& a, int total_chunks, hipStream_t s) {
    if (a.nframes <= 0 || total_chunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_chunk_scan<true>, dim3(a.nframes), dim3(SNT), 0, s, a);
    hipLaunchKernelGGL(k_stream_offsets, dim3(1), dim3(64), 0, s, a);
    hipLaunchKernelGGL(k_encode_chunk, dim3(total_chunks), dim3(CNT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_ridge_decode(const RidgeCodeArgs& a, int total_chunks, hipStream_t s) {
    if (a.nframes <= 0 || total_chunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_chunk_scan<false>, dim3(a.nframes), dim3(SNT), 0, s, a);
    hipLaunchKernelGGL(k_decode_chunk, dim3(total_chunks), dim3(CNT), 0, s, a);
    return hipGetLastError();
}

}  // namespace rd
