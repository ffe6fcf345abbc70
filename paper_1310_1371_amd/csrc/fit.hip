// Ridge classification and sub-pixel circle fit (method step 5).
//
// One workgroup per peak (a, b, r): it visits the 16x16 ridge bins that overlap the
// annulus' bounding box, takes the ridge pixels with (max(r-w,0))^2 <= (x-a)^2 + (y-b)^2
// <= (r+w)^2 (an exact integer test; a ridge pixel may belong to several peaks), sums the
// nine normal-equation moments of the algebraic (Kasa) fit exactly in int64, and one thread
// solves the 3x3 system in fp64.  The workgroup also counts the frame's peaks that precede
// its own in (r, b, a) order and writes the ring at that rank: peaks are distinct voxels, so
// the ranks are a permutation and every frame's ring list comes out sorted.
#include "rd_internal.h"

namespace rd {
namespace {

__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Solve M x = rhs (3x3) by Gaussian elimination with partial pivoting.  Returns false if
// a pivot is exactly zero.
__device__ bool solve3(double M[3][3], double rhs[3], double x[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        int p = c;
        for (int r = c + 1; r < 3; ++r)
            if (fabs(M[r][c]) > fabs(M[p][c])) p = r;
        if (M[p][c] == 0.0) return false;
        if (p != c) {
            for (int k = 0; k < 3; ++k) {
                const double t = M[c][k]; M[c][k] = M[p][k]; M[p][k] = t;
            }
            const double t = rhs[c]; rhs[c] = rhs[p]; rhs[p] = t;
        }
        for (int r = c + 1; r < 3; ++r) {
            const double f = M[r][c] / M[c][c];
            for (int k = c; k < 3; ++k) M[r][k] -= f * M[c][k];
            rhs[r] -= f * rhs[c];
        }
    }
    for (int c = 2; c >= 0; --c) {
        double s = rhs[c];
        for (int k = c + 1; k < 3; ++k) s -= M[c][k] * x[k];
        x[c] = s / M[c][c];
    }
    return true;
}

constexpr int FNT = 256;   // threads per peak

// Exclusive prefix over the block; *total receives the sum.  Contains __syncthreads.
__device__ __forceinline__ uint32_t fit_excl_scan(uint32_t v, uint32_t* s_wave, uint32_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t n = __shfl_up(inc, o, 64);
        if (lane >= o) inc += n;
    }
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < FNT / 64; ++w) {
        if (w < wave) base += s_wave[w];
        tot += s_wave[w];
    }
    *total = tot;
    return base + inc - v;
}

// One workgroup per peak.  The ridge slots of the bins in the annulus' bounding box are
// flattened (a prefix over the bin counts, up to FNT bins per round) so that every thread
// issues independent loads; the nine moments are summed per thread, then per wave, then
// over the workgroup.
__global__ __launch_bounds__(FNT) void k_fit(FitArgs a) {
    __shared__ uint32_t sPre[FNT + 1];
    __shared__ int64_t sBinBase[FNT];
    __shared__ uint32_t sWave[FNT / 64];
    __shared__ int64_t sMom[FNT / 64][10];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (blockIdx.x == 0 && tid == 0 && a.counts_out) {
        for (int f = 0; f < a.nframes; ++f) a.counts_out[f] = a.peak_count[f];
        a.counts_out[a.nframes] = a.error ? *a.error : 0u;
    }
    if (blockIdx.x == 0 && a.stats_out)                      // the earlier kernels have finished
        for (int i = tid; i < a.nstats; i += FNT) a.stats_out[i] = a.stats_in[i];
    for (int f = 0; f < a.nframes; ++f) {
        const FrameDesc fd = a.frames[f];
        const uint32_t np = min(a.peak_count[f], static_cast<uint32_t>(a.max_peaks));
        for (uint32_t p = blockIdx.x; p < np; p += gridDim.x) {
            const Peak pk = a.peaks[fd.peak0 + p];
            const int pa = pk.a, pb = pk.b, r = pk.r;
            const int ro = r + a.w, ri = max(r - a.w, 0);
            const int64_t ro2 = static_cast<int64_t>(ro) * ro, ri2 = static_cast<int64_t>(ri) * ri;
            const int bxlo = max((pa - ro) >> BIN_SHIFT, 0), bxhi = min((pa + ro) >> BIN_SHIFT, fd.nbx - 1);
            const int bylo = max((pb - ro) >> BIN_SHIFT, 0), byhi = min((pb + ro) >> BIN_SHIFT, fd.nby - 1);
            // n, su, sv, suu, suv, svv, sz, suz, svz, and the rank of the peak in its frame
            int64_t m[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
            for (uint32_t q = tid; q < np; q += FNT) {
                const Peak o = a.peaks[fd.peak0 + q];
                m[9] += (o.r < r || (o.r == r && (o.b < pb || (o.b == pb && o.a < pa)))) ? 1 : 0;
            }
            const int nbxr = bxhi - bxlo + 1;
            const int nbin = nbxr * (byhi - bylo + 1);
            for (int b0 = 0; b0 < nbin; b0 += FNT) {       // rounds of up to FNT bins
                const int bi = b0 + tid;
                uint32_t cnt = 0;
                int64_t bin = 0;
                if (bi < nbin) {
                    const int by = bylo + bi / nbxr, bx = bxlo + bi % nbxr;
                    bin = fd.bin0 + static_cast<int64_t>(by) * fd.nbx + bx;
                    cnt = min(a.bin_count[bin], static_cast<uint32_t>(BIN_CAP));
                }
                uint32_t total;
                const uint32_t pre = fit_excl_scan(cnt, sWave, &total);
                sPre[tid] = pre;
                sBinBase[tid] = bin * BIN_CAP;
                if (tid == 0) sPre[FNT] = total;
                __syncthreads();
                for (uint32_t k = tid; k < total; k += FNT) {
                    int lo = 0, hi = FNT;                   // largest lo with sPre[lo] <= k
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (sPre[mid] <= k) lo = mid; else hi = mid;
                    }
                    const uint32_t xy = a.rxy[sBinBase[lo] + (k - sPre[lo])];
                    const int64_t u = static_cast<int>(xy & 0xffffu) - pa;
                    const int64_t v = static_cast<int>(xy >> 16) - pb;
                    const int64_t z = u * u + v * v;
                    if (z >= ri2 && z <= ro2) {
                        m[0] += 1; m[1] += u; m[2] += v; m[3] += u * u; m[4] += u * v; m[5] += v * v;
                        m[6] += z; m[7] += u * z; m[8] += v * z;
                    }
                }
                __syncthreads();                              // sPre is rewritten next round
            }
#pragma unroll
            for (int i = 0; i < 10; ++i) m[i] = wave_sum64(m[i]);
            if (lane == 0)
#pragma unroll
                for (int i = 0; i < 10; ++i) sMom[wave][i] = m[i];
            __syncthreads();
            if (tid == 0) {
#pragma unroll
                for (int i = 0; i < 10; ++i) {
                    m[i] = sMom[0][i];
                    for (int w = 1; w < FNT / 64; ++w) m[i] += sMom[w][i];
                }
                const int64_t n = m[0], su = m[1], sv = m[2], suu = m[3], suv = m[4], svv = m[5];
                const int64_t sz = m[6], suz = m[7], svz = m[8];
                double cx = pa, cy = pb, rr = r;
                int ok = 0;
                if (n >= a.min_pts) {
                    double M[3][3] = {{(double)suu, (double)suv, (double)su},
                                      {(double)suv, (double)svv, (double)sv},
                                      {(double)su, (double)sv, (double)n}};
                    double rhs[3] = {-(double)suz, -(double)svz, -(double)sz};
                    double sol[3];
                    if (solve3(M, rhs, sol)) {
                        const double ccx = pa - 0.5 * sol[0], ccy = pb - 0.5 * sol[1];
                        const double r2 = 0.25 * sol[0] * sol[0] + 0.25 * sol[1] * sol[1] - sol[2];
                        if (isfinite(ccx) && isfinite(ccy) && isfinite(r2) && r2 >= 0.0) {
                            const double rf = sqrt(r2);
                            if (hypot(ccx - pa, ccy - pb) <= a.w && fabs(rf - r) <= a.w) {
                                cx = ccx; cy = ccy; rr = rf; ok = 1;
                            }
                        }
                    }
                }
                rd_ring ring;
                ring.cx = static_cast<float>(cx);
                ring.cy = static_cast<float>(cy);
                ring.r = static_cast<float>(rr);
                ring.score = static_cast<float>(static_cast<double>(pk.s) / (static_cast<double>(r) * 1073741824.0));
                ring.a = pa; ring.b = pb; ring.r_bin = r;
                ring.n_fit = static_cast<int32_t>(n);
                ring.fit_ok = ok;
                a.rings[fd.peak0 + m[9]] = ring;    // 0 <= rank < np
            }
            __syncthreads();                                  // sMom is rewritten by the next peak
        }
    }
}

}  // namespace

hipError_t launch_fit(const FitArgs& a, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_fit, dim3(blocks), dim3(FNT), 0, s, a);
    return hipGetLastError();
}

}  // namespace rd
