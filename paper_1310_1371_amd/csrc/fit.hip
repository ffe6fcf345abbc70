// Ridge classification and sub-pixel circle fit (method step 5).
//
// One wavefront per peak (a, b, r): it visits the 16x16 ridge bins that overlap the
// annulus' bounding box, takes the ridge pixels with (max(r-w,0))^2 <= (x-a)^2 + (y-b)^2
// <= (r+w)^2 (an exact integer test; a ridge pixel may belong to several peaks), sums the
// nine normal-equation moments of the algebraic (Kasa) fit exactly in int64, and lane 0
// solves the 3x3 system in fp64.
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

__global__ __launch_bounds__(64) void k_fit(FitArgs a) {
    const int lane = threadIdx.x;
    if (blockIdx.x == 0 && lane == 0 && a.counts_out) {
        for (int f = 0; f < a.nframes; ++f) a.counts_out[f] = a.peak_count[f];
        a.counts_out[a.nframes] = a.error ? *a.error : 0u;
    }
    for (int f = 0; f < a.nframes; ++f) {
        const FrameDesc fd = a.frames[f];
        const uint32_t np = min(a.peak_count[f], static_cast<uint32_t>(a.max_peaks));
        for (uint32_t p = blockIdx.x; p < np; p += gridDim.x) {
            const Peak pk = a.peaks[fd.peak0 + p];
            const int pa = pk.a, pb = pk.b, r = pk.r;
            const int ro = r + a.w, ri = max(r - a.w, 0);
            const int ro2 = ro * ro, ri2 = ri * ri;
            const int bxlo = max((pa - ro) >> BIN_SHIFT, 0), bxhi = min((pa + ro) >> BIN_SHIFT, fd.nbx - 1);
            const int bylo = max((pb - ro) >> BIN_SHIFT, 0), byhi = min((pb + ro) >> BIN_SHIFT, fd.nby - 1);
            int64_t n = 0, su = 0, sv = 0, suu = 0, suv = 0, svv = 0, sz = 0, suz = 0, svz = 0;
            const int nbxr = bxhi - bxlo + 1;
            const int nbin = nbxr * (byhi - bylo + 1);
            for (int bi = lane; bi < nbin; bi += 64) {     // one bin per lane
                const int by = bylo + bi / nbxr, bx = bxlo + bi % nbxr;
                const int64_t bin = fd.bin0 + (int64_t)by * fd.nbx + bx;
                const uint32_t cnt = min(a.bin_count[bin], static_cast<uint32_t>(BIN_CAP));
                for (uint32_t i = 0; i < cnt; ++i) {
                    const uint32_t xy = a.rxy[bin * BIN_CAP + i];
                    const int64_t u = static_cast<int>(xy & 0xffffu) - pa;
                    const int64_t v = static_cast<int>(xy >> 16) - pb;
                    const int64_t z = u * u + v * v;
                    if (z >= ri2 && z <= ro2) {
                        n += 1; su += u; sv += v; suu += u * u; suv += u * v; svv += v * v;
                        sz += z; suz += u * z; svz += v * z;
                    }
                }
            }
            n = wave_sum64(n); su = wave_sum64(su); sv = wave_sum64(sv);
            suu = wave_sum64(suu); suv = wave_sum64(suv); svv = wave_sum64(svv);
            sz = wave_sum64(sz); suz = wave_sum64(suz); svz = wave_sum64(svz);
            if (lane == 0) {
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
                a.rings[fd.peak0 + p] = ring;
            }
        }
    }
}

}  // namespace

hipError_t launch_fit(const FitArgs& a, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_fit, dim3(blocks), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace rd
