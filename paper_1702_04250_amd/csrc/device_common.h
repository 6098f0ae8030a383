// Device-side helpers shared by the kernels of the MI355X PPPM library.
#pragma once

#include <hip/hip_runtime.h>

#include "pppm_internal.h"

namespace pppm {

// Number of XCDs (chiplets, each with its own L2) of an MI355X.  Workgroups
// are handed to XCDs round-robin (workgroup i to XCD i mod 8).  The remap
// gives each XCD runs of XCD_CHUNK consecutive tiles (neighbours along x,
// which share halo records in that XCD's L2), and deals the runs to the XCDs
// round-robin, so every XCD's share is spread over the whole mesh and a
// charge density that varies across the box still loads the XCDs evenly.
// The tail that does not fill a whole round keeps the identity order.
constexpr int NUM_XCD = 8;
constexpr int XCD_CHUNK = 4;

template <int CHUNK = XCD_CHUNK>
__device__ __forceinline__ int xcd_remap(int wg, int nwg)
{
    constexpr int ROUND = NUM_XCD * CHUNK;
    const int nfull = nwg / ROUND * ROUND;
    if (wg >= nfull) return wg;
    const int x = wg % NUM_XCD, local = wg / NUM_XCD;
    return (local / CHUNK) * ROUND + x * CHUNK + local % CHUNK;
}

// Deals the workgroups to the XCDs in NUM_XCD contiguous runs: XCD x takes
// logical workgroups [x * per, (x + 1) * per), per = nwg / NUM_XCD.  The
// tail that does not fill a run keeps the identity order.
__device__ __forceinline__ int xcd_contiguous(int wg, int nwg)
{
    const int per = nwg / NUM_XCD;
    if (wg >= per * NUM_XCD) return wg;
    return (wg % NUM_XCD) * per + wg / NUM_XCD;
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

// Stencil weights of one axis as polynomials.  On a stencil the weight of
// point s + j is w_j(f) = M_P(f + P - 1 - j), M_P the cardinal B-spline of
// order P, a polynomial of degree P - 1 in the fraction f.  Its coefficients
// in g = f - 1/2 (exact rationals, from the two-term B-spline recursion
// applied to the polynomial pieces) are c[j][m], w_j = sum_m c[j][m] g^m.
// Centring on g keeps every power below 1/2 in size, so Horner's rule loses
// no accuracy near either end of the cell.  Mirror symmetry,
// w_{P-1-j}(g) = w_j(-g), leaves only the rows j <= (P - 1) / 2.
template <int P> struct WeightPoly;
template <> struct WeightPoly<2> {
    static constexpr double c[1][2] = {{1.0 / 2, -1.0}};
};
template <> struct WeightPoly<3> {
    static constexpr double c[2][3] = {{1.0 / 8, -1.0 / 2, 1.0 / 2}, {3.0 / 4, 0.0, -1.0}};
};
template <> struct WeightPoly<4> {
    static constexpr double c[2][4] = {{1.0 / 48, -1.0 / 8, 1.0 / 4, -1.0 / 6},
                                       {23.0 / 48, -5.0 / 8, -1.0 / 4, 1.0 / 2}};
};
template <> struct WeightPoly<5> {
    static constexpr double c[3][5] = {{1.0 / 384, -1.0 / 48, 1.0 / 16, -1.0 / 12, 1.0 / 24},
                                       {19.0 / 96, -11.0 / 24, 1.0 / 4, 1.0 / 6, -1.0 / 6},
                                       {115.0 / 192, 0.0, -5.0 / 8, 0.0, 1.0 / 4}};
};
template <> struct WeightPoly<6> {
    static constexpr double c[3][6] = {
        {1.0 / 3840, -1.0 / 384, 1.0 / 96, -1.0 / 48, 1.0 / 48, -1.0 / 120},
        {79.0 / 1280, -25.0 / 128, 7.0 / 32, -1.0 / 16, -1.0 / 16, 1.0 / 24},
        {841.0 / 1920, -77.0 / 192, -11.0 / 48, 7.0 / 24, 1.0 / 24, -1.0 / 12}};
};
template <> struct WeightPoly<7> {
    static constexpr double c[4][7] = {
        {1.0 / 46080, -1.0 / 3840, 1.0 / 768, -1.0 / 288, 1.0 / 192, -1.0 / 240, 1.0 / 720},
        {361.0 / 23040, -59.0 / 960, 37.0 / 384, -5.0 / 72, 1.0 / 96, 1.0 / 60, -1.0 / 120},
        {10543.0 / 46080, -289.0 / 768, 79.0 / 768, 43.0 / 288, -17.0 / 192, -1.0 / 48, 1.0 / 48},
        {5887.0 / 11520, 0.0, -77.0 / 192, 0.0, 7.0 / 48, 0.0, -1.0 / 36}};
};

// w[j] = w_j(f) and, with DERIV, dw[j] = d w_j / df = M_{P-1}(f + P - 1 - j)
// - M_{P-1}(f + P - 2 - j) (the derivative along the axis in mesh units).
// Each mirror pair is evaluated from its even and odd parts in g:
// w_j = E + g O, w_{P-1-j} = E - g O; dw_j = D + g Q, dw_{P-1-j} = g Q - D.
template <int P, typename R, bool DERIV>
__device__ __forceinline__ void bspline(R f, R (&w)[P], R (&dw)[P])
{
    using C = WeightPoly<P>;
    const R g = f - R(0.5), g2 = g * g;
#pragma unroll
    for (int j = 0; j < (P + 1) / 2; ++j) {
        R e = R(0), o = R(0);
#pragma unroll
        for (int m = P - 1; m >= 0; --m) {
            if (m % 2 == 0) e = e * g2 + R(C::c[j][m]);
            else o = o * g2 + R(C::c[j][m]);
        }
        w[j] = e + g * o;
        if (P - 1 - j != j) w[P - 1 - j] = e - g * o;
        if (DERIV) {
            // derivative coefficients (m + 1) c[j][m + 1], m = 0 .. P - 2
            R de = R(0), dq = R(0);
#pragma unroll
            for (int m = P - 2; m >= 0; --m) {
                if (m % 2 == 0) de = de * g2 + R((m + 1) * C::c[j][m + 1]);
                else dq = dq * g2 + R((m + 1) * C::c[j][m + 1]);
            }
            dw[j] = de + g * dq;
            if (P - 1 - j != j) dw[P - 1 - j] = g * dq - de;
        }
    }
}

// Stencil weights of one axis from the polynomials or, when the plan carries
// a table (the tabulated variant of the mapping functions, paper Section
// 3.1), from its nearest entry: T + 1 rows at f = i / T, each the P weights
// followed by the P derivative weights.
template <int P, typename R, bool DERIV, bool TAB>
__device__ __forceinline__ void stencil_weights(R f, const MapGeo& g, R (&w)[P], R (&dw)[P])
{
    if constexpr (TAB) {
        int i = (int)(f * (R)g.wtab_n + R(0.5));
        i = i < 0 ? 0 : (i > g.wtab_n ? g.wtab_n : i);
        const R* row = (const R*)g.wtab + (size_t)i * (2 * P);
#pragma unroll
        for (int j = 0; j < P; ++j) {
            w[j] = row[j];
            if (DERIV) dw[j] = row[P + j];
        }
    } else {
        bspline<P, R, DERIV>(f, w, dw);
    }
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
