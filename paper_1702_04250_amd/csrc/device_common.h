// Device-side helpers shared by the kernels of the MI355X PPPM library.
#pragma once

#include <hip/hip_runtime.h>

#include "pppm_internal.h"

namespace pppm {

// Number of XCDs (chiplets, each with its own L2) of an MI355X.  Workgroups
// are handed to XCDs round-robin; remapping gives each XCD one contiguous
// slab of tiles so neighbouring tiles share halo data in the same L2.
constexpr int NUM_XCD = 8;

__device__ __forceinline__ int xcd_remap(int wg, int nwg)
{
    const int q = nwg / NUM_XCD, r = nwg % NUM_XCD;
    const int x = wg % NUM_XCD, local = wg / NUM_XCD;
    return x * q + (x < r ? x : r) + local;
}

// Record of a binned particle: stencil start within its tile plus the
// fraction (t in [0, B]) per axis, and the charge.
template <typename R> struct Rec;
template <> struct Rec<float> { using T = float4; };
template <> struct Rec<double> { using T = double4; };

// Periodic map of one coordinate to its stencil start.  u = (x - lo) / h is
// wrapped into [0, K); the stencil start is s = floor(u + 1 - P/2) taken
// modulo K and the fraction is f = u + 1 - P/2 - floor(u + 1 - P/2).
// Returns false (and maps to u = 0) for a non-finite or unrepresentable x.
__device__ __forceinline__ bool map_coord(double x, double lo, double h, int K, double shift,
                                          int& s_mod, double& f)
{
    // Plain IEEE operations, no fused multiply-add: the integer decision s is
    // taken exactly as a straightforward FP64 evaluation takes it.
#pragma clang fp contract(off)
    const double Kd = (double)K;
    double u = (x - lo) / h;
    u = u - Kd * floor(u / Kd);
    if (u < 0.0) u += Kd;
    if (u >= Kd) u -= Kd;
    bool ok = (u >= 0.0) && (u < Kd);  // false for NaN / Inf / huge |x|
    if (!ok) u = 0.0;
    const double t = u + shift;
    const double s = floor(t);
    f = t - s;
    int si = (int)s;          // in [floor(shift), K - 1]
    if (si < 0) si += K;
    if (si >= K) si -= K;
    s_mod = si;
    return ok;
}

// Cardinal B-spline stencil of one axis.  a[k] after building order n holds
// M_n(f + k); the two-term recursion M_n(x) = [x M_{n-1}(x) + (n - x)
// M_{n-1}(x - 1)] / (n - 1) is evaluated for the P offsets at once.
// w[j] = M_P(f + P - 1 - j) is the weight of stencil point s + j and
// dw[j] = M_{P-1}(f + P - 1 - j) - M_{P-1}(f + P - 2 - j) its d/du.
template <int P, typename R, bool DERIV>
__device__ __forceinline__ void bspline(R f, R (&w)[P], R (&dw)[P])
{
    R a[P];
    a[0] = R(1);
#pragma unroll
    for (int k = 1; k < P; ++k) a[k] = R(0);
#pragma unroll
    for (int m = 2; m <= P; ++m) {
        if (DERIV && m == P) {
#pragma unroll
            for (int j = 0; j < P; ++j) {
                const int k1 = P - 1 - j, k2 = P - 2 - j;
                const R hi = (k1 <= P - 2) ? a[k1] : R(0);
                const R lo = (k2 >= 0) ? a[k2] : R(0);
                dw[j] = hi - lo;
            }
        }
        const R inv = R(1) / R(m - 1);
        R next[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            if (k < m) {
                const R left = (k < m - 1) ? a[k] : R(0);
                const R right = (k >= 1) ? a[k - 1] : R(0);
                next[k] = ((f + R(k)) * left + (R(m) - f - R(k)) * right) * inv;
            } else {
                next[k] = R(0);
            }
        }
#pragma unroll
        for (int k = 0; k < P; ++k) a[k] = next[k];
    }
#pragma unroll
    for (int j = 0; j < P; ++j) w[j] = a[P - 1 - j];
}

// Inclusive warp-level scan over a 64-wide wavefront.
__device__ __forceinline__ int wave_inclusive_scan(int v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// Exclusive scan of one int per thread over the whole workgroup (blockDim a
// multiple of 64, at most 1024).  Returns the exclusive prefix; *total gets
// the sum.  Uses shared scratch of 17 ints.
__device__ __forceinline__ int block_exclusive_scan(int v, int* scratch, int* total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    int inc = wave_inclusive_scan(v);
    if (lane == 63) scratch[wid] = inc;
    __syncthreads();
    if (wid == 0) {
        int x = lane < nw ? scratch[lane] : 0;
        int xi = wave_inclusive_scan(x);
        if (lane < nw) scratch[lane] = xi - x;
        if (lane == nw - 1) scratch[16] = xi;
    }
    __syncthreads();
    int res = inc - v + scratch[wid];
    *total = scratch[16];
    __syncthreads();
    return res;
}

}  // namespace pppm
