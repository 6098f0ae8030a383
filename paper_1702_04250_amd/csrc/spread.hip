// make_rho: the paper's Map-Charge (Section 3.1).  Each charge adds
// q * wx * wy * wz to the P^3 mesh points of its stencil.
//
// GPU design (owner computes): one workgroup owns one tile of mesh points and
// accumulates it in LDS.  It reads every binned charge whose stencil reaches
// into the tile - the charges of the tile's own sub-bricks and those of the
// sub-bricks up to P - 1 points below it - and adds the part of each stencil
// that falls inside the tile with LDS atomics.  Every mesh point is owned by
// exactly one tile, so the tile is flushed to the global mesh with plain
// coalesced stores: no global atomics and no zero-fill of the mesh.
// This is the GPU counterpart of the paper's per-thread private grids
// ("rethread"): privatise, accumulate, then combine - here the combine is a
// disjoint ownership of the output.  At P >= 6 (and at P = 5 when the tiles
// are fewer than the CUs) the mixed form takes the push form instead
// (k_spread_push + k_fold, below): each tile sums only its own charges,
// whole stencils, and a fold kernel combines the overlapping tiles.
//
// Accumulator.  On gfx950 the LDS float atomic add (ds_add_f32) is processed
// at about one lane every three clocks for any non-uniform address pattern,
// some 30x slower than the integer one (ds_add_u32).  The mixed-precision
// form therefore accumulates each tile in exact 32-bit fixed point: every
// FP32 contribution q wx wy wz is rounded to an integer multiple of 2^-e and
// added with ds_add_u32.  Integer addition is associative (modulo 2^32), so
// the sum is exact and independent of the order of the atomics, and it is
// correct whenever the final value fits, |rho_m| 2^e < 2^31 (intermediate
// sums may wrap).  e is chosen per tile from a bound on any of its points:
// a charge adds at most max|q| wmax(P)^3 to a point, and only charges whose
// stencil starts within P - 1 points below it reach it.  A first pass counts
// the tile's charges per coarse cell of 4^3 stencil starts; the bound of a
// point is then that count summed over the cells that can hold the starts
// of its covering stencils, times max|q| wmax^3, with one bit of headroom.
// At the mean density of the benchmark systems this is about eight times
// finer than bounding by all the charges the tile reads.  A tile that reads
// more than WIDE_VISITS charges (a dense cluster) skips the count and sums
// the same 32-bit rounded contributions in 64 bits (ds_add_u64), with the
// unit set by the largest single contribution; so does a tile whose reach
// bound exceeds WIDE_REACH, and every tile when the largest |q| exceeds
// WIDE_RANGE times the RMS |q| of all the charges.
// The rounding is unbiased: each contribution v is rounded to floor(v + d)
// with a dither d in [0, 1) that is a hash of the charge's record and of the
// stencil point, so its expectation is v.  Rounding to nearest instead sends
// every contribution smaller than half a unit to zero; the far corners of
// the stencils are such contributions for every charge alike, so each
// charge's mesh cloud loses the same sliver of charge, and the mesh energy,
// which sums q_i^2 times each cloud's self-interaction, moves coherently
// over all charges (by 1.2e-5 of E on 524,288 +-1 charges at 128^3, P = 5,
// where E_mesh and E_self cancel to 1/15).  With the dither the errors are
// zero-mean and average out over the charges.  The dither depends only on
// the record's bits (position within the tile and charge), so the sum stays
// independent of the order of the charges.  The flush
// converts each exact sum to FP64; that value goes to the caller's FP64 mesh
// when one is asked for, and, rounded to FP32, to the plan's FFT input (the
// mixed form transforms in FP32).  The FP64 form does the same in 64-bit
// fixed point (FP64 products rounded to integers, ds_add_u64, 2^62 bound):
// faster than ds_add_f64 and, like the mixed form, independent of the order
// of the atomics; it keeps an FP64 FFT input.
#include <algorithm>

#include "tiles.h"

namespace pppm {

namespace {

struct SpreadArgs {
    MapGeo g;
    const int* offsets;
    const void* rec;
    void* rho;            // plan mesh of type R (the FFT input)
    double* rho_user;     // caller's FP64 mesh or null
    const double* stats;  // [1] max |q|, [2] sum q^2 (from the particle map)
    int pitch_x;          // LDS row pitch (points): B_x + 2 (P - 1)
    int rows_y;           // LDS rows per plane: B_y, + P - 1 on a single-tile axis
    int planes_z;         // LDS planes: B_z, + P - 1 on a single-tile axis
    int occ_off;          // byte offset of the occupancy count in LDS
    int occ_shift[3];     // log2 of the coarse cell edge per axis (mesh points)
    int occ_n[3];         // coarse cells per axis
    int occ_k[3];         // cells below a point's cell that its covering stencils can start in
    float* box;           // push form: [ntiles][box_stride] FP32 partial sums of each tile's box
    int box_stride;       // points of one box: box_pitch * box_rows * box_planes
    int box_pitch;        // B_x + P - 1
    int box_rows;         // B_y + P - 1
    int box_planes;       // B_z + P - 1
};

// Largest value of the order-P B-spline (P = 2..7), rounded up.
__host__ __device__ constexpr double bspline_max(int P)
{
    return P == 2 ? 1.0 : P == 3 ? 0.7501 : P == 4 ? 0.6668 : P == 5 ? 0.5991 : P == 6 ? 0.5501 : 0.5111;
}

// Fixed-point exponent for a BITS-bit accumulator when at most `visits`
// charges reach any point (see above): the bound times 2^e stays below
// 2^(BITS - 2), one bit of headroom.  In a sparse tile single contributions
// may reach 2^30 units; from 2^24 units on the FP32 value v is an integer
// and v + d rounds back to v, so such a contribution is added exactly as
// the FP32 product (no fixed-point rounding at all).
template <int P, int BITS>
__device__ __forceinline__ int fixed_point_exponent(int visits, double qmax)
{
    const double wm = bspline_max(P);
    const double bound = (double)visits * qmax * wm * wm * wm;
    if (!(bound > 0.0)) return BITS - 2;
    const int e = (int)floor(log2(ldexp(1.0, BITS - 2) / bound));
    return e < -60 ? -60 : (e > 120 ? 120 : e);
}

// Mixed form, dense tiles: above WIDE_VISITS charges the 32-bit bound would
// round too coarsely (the unit grows with the visits while a point's charge
// grows about as their square root), so such a tile sums in 64 bits and the
// exponent only has to keep one contribution (a 32-bit integer) below 2^30
// units; the sum of at most 2^31 of them stays far inside 2^63.
constexpr int WIDE_VISITS = 8192;
// ... and so does every tile when the charges span a wide range of
// magnitudes: the 32-bit unit follows the largest |q|, so when that exceeds
// WIDE_RANGE times the RMS |q| of all charges the typical contribution
// would be resolved coarsely (molecular charges stay near 1, Gaussian ones
// below 6 up to millions of charges).
constexpr double WIDE_RANGE = 8.0;
// ... and so does a tile whose reach bound (the most charges that can reach
// one of its points) exceeds WIDE_REACH: the 32-bit unit grows with the
// bound while the resolution a point needs does not (at 26 charges per mesh
// point the 32-bit sums held the mesh charge only to 1.3e-4; at two
// charges per point, P = 5, to 2.0e-5, where the 64-bit sums reach 5.3e-7
// for 2.5 % more time).  The benchmark systems reach about 130.
constexpr int WIDE_REACH = 512;
__device__ __forceinline__ bool wide_charge_range(const SpreadArgs& a)
{
    const MapGeo& g = a.g;
    const int n = a.offsets[g.ntiles * NCLASS * g.bin_stride];
    return n > 0 && a.stats[1] * a.stats[1] * n > WIDE_RANGE * WIDE_RANGE * a.stats[2];
}
template <int P>
__device__ __forceinline__ int contribution_exponent(double qmax)
{
    const double wm = bspline_max(P);
    const double one = qmax * wm * wm * wm;
    if (!(one > 0.0)) return 30;
    const int e = (int)floor(log2(ldexp(1.0, 30) / one));
    return e < -60 ? -60 : (e > 120 ? 120 : e);
}

// Dither of the rounding: a 24-bit hash of the record's four words, as a
// fraction in [0, 1); the rows of the stencil then take the Weyl sequence
// d + jy a2 + jz a3 (mod 1) with steps of the 2-D R2 low-discrepancy
// sequence (powers of the inverse of the plastic number, g^3 = g + 1), so
// every row's dither is uniform on [0, 1).  The points of a row share their
// row's dither: each contribution is still rounded without bias, and the
// dither costs one add and one fract per row rather than per point.
__device__ __forceinline__ float dither_seed(float4 r)
{
    unsigned h = __float_as_uint(r.x) * 0x9E3779B1u;
    h ^= __float_as_uint(r.y) * 0x85EBCA77u;
    h ^= __float_as_uint(r.z) * 0xC2B2AE3Du;
    h ^= __float_as_uint(r.w) * 0x27D4EB2Fu;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    return (float)(h >> 8) * 0x1p-24f;
}
__device__ __forceinline__ float dither_seed(double4) { return 0.0f; }
constexpr float DITHER_Y = 0.7548776662f, DITHER_Z = 0.5698402910f;

// Adds the contribution a * b (already scaled by 2^e) with dither d.
template <typename A> struct Acc;
template <> struct Acc<int> {
    // floor(a b + d): one fused multiply-add and v_cvt_flr_i32_f32
    __device__ static void add(int* p, float a, float b, float d)
    {
        const float v = __builtin_fmaf(a, b, d);
        int r;
        asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(v));
        atomicAdd(p, r);
    }
};
template <> struct Acc<long long> {
    // FP64 form: 64-bit fixed point, the product rounded to nearest (its
    // unit, 2^-e with e near 53 for the benchmark systems, is far below the
    // FP64 rounding of the products, so no dither is needed)
    __device__ static void add(long long* p, double a, double b, float)
    {
        atomicAdd((unsigned long long*)p, (unsigned long long)__double2ll_rn(a * b));
    }
    // mixed form, dense tile: the same 32-bit dithered rounding, summed in
    // 64 bits
    __device__ static void add(long long* p, float a, float b, float d)
    {
        const float v = __builtin_fmaf(a, b, d);
        int r;
        asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(v));
        atomicAdd((unsigned long long*)p, (unsigned long long)(long long)r);
    }
};
__device__ __forceinline__ float fract1(float x) { return __builtin_amdgcn_fractf(x); }

// Tile coordinate of the stencil start of a record read through run r.
template <typename RT>
__device__ __forceinline__ void stencil_start(const RunTable& rt, int r, const RT& c, int (&dd)[3])
{
    const int shp = rt.shift[r], exp_ = rt.ext[r];
    const decltype(c.x) tt[3] = {c.x, c.y, c.z};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        int sl;
        decltype(c.x) f;
        decode_local(tt[d], (exp_ >> (8 * d)) & 255, sl, f);
        dd[d] = sl + ((shp >> (8 * d)) & 255) - 128;  // in [-H, ext)
    }
}

// Most charges whose stencils can reach any one point of the tile, from the
// count per coarse cell of stencil starts: a point's count is the sum over
// the cells from occ_k below its own cell up to it along each axis (a
// stencil reaching the point starts at most P - 1 points below it).  Adds
// the block's maximum to wmax[wave]; the caller synchronises.
__device__ __forceinline__ void reach_bound(const SpreadArgs& a, const int* occ, const int (&ext)[3], int* wmax)
{
    const int H = a.g.halo;
    int c0[3], nc[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        c0[d] = min(H >> a.occ_shift[d], a.occ_n[d] - 1);
        nc[d] = min((ext[d] - 1 + H) >> a.occ_shift[d], a.occ_n[d] - 1) - c0[d] + 1;
    }
    int best = 0;
    for (int i = threadIdx.x; i < nc[0] * nc[1] * nc[2]; i += blockDim.x) {
        const int cx = c0[0] + i % nc[0], cy = c0[1] + (i / nc[0]) % nc[1], cz = c0[2] + i / (nc[0] * nc[1]);
        int sum = 0;
        for (int z = max(0, cz - a.occ_k[2]); z <= cz; ++z)
            for (int y = max(0, cy - a.occ_k[1]); y <= cy; ++y)
                for (int x = max(0, cx - a.occ_k[0]); x <= cx; ++x) sum += occ[(z * a.occ_n[1] + y) * a.occ_n[0] + x];
        best = max(best, sum);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) best = max(best, __shfl_xor(best, o, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = best;
}

__device__ __forceinline__ int occ_cell(const SpreadArgs& a, const int (&dd)[3])
{
    const int H = a.g.halo;
    int c[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) c[d] = min((dd[d] + H) >> a.occ_shift[d], a.occ_n[d] - 1);
    return (c[2] * a.occ_n[1] + c[1]) * a.occ_n[0] + c[0];
}

// First pass of a 32-bit mixed-form tile whose visits are taken in binned
// order: the occupancy count and the reach bound.  Ends synchronised.
template <typename RT>
__device__ __forceinline__ int count_pass(const SpreadArgs& a, const RunTable& rt, int* occ, int* wmax, RT cur,
                                          int nown, const int (&ext)[3])
{
    const RT* __restrict__ rec = (const RT*)a.rec;
    const int total = rt.pre[NRUNS];
    for (int v = threadIdx.x; v < total; v += blockDim.x) {
        const int r = find_run(rt, v);
        if (v >= nown || v != (int)threadIdx.x) cur = rec[rt.start[r] + (v - rt.pre[r])];
        int dd[3];
        stencil_start(rt, r, cur, dd);
        atomicAdd(&occ[occ_cell(a, dd)], 1);
    }
    __syncthreads();
    reach_bound(a, occ, ext, wmax);
    __syncthreads();
    int reach = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) reach = max(reach, wmax[w]);
    return reach;
}

// The visits of one tile, the periodic folds and the flush, with accumulator
// type AC (int: 32-bit fixed point; long long: 64-bit) and unit 2^-e.
template <int P, typename R, typename AC, bool TAB>
__device__ __forceinline__ void spread_tile(const SpreadArgs& a, const RunTable& rt, AC* acc, int e,
                                            typename Rec<R>::T cur, int nown, const int (&T0)[3],
                                            const int (&ext)[3])
{
    const MapGeo& g = a.g;
    constexpr int H = P - 1;
    using RT = typename Rec<R>::T;
    const RT* __restrict__ rec = (const RT*)a.rec;
    const int pitch = a.pitch_x;
    const int plane = pitch * a.rows_y;
    const int total = rt.pre[NRUNS];
    const R scale = (R)ldexp(1.0, e);
    // valid y rows / z planes: [0, lim)
    const int lim_y = g.ntile[1] == 1 ? g.K[1] + H : ext[1];
    const int lim_z = g.ntile[2] == 1 ? g.K[2] + H : ext[2];

    for (int v = threadIdx.x; v < total; v += blockDim.x) {
        const int r = find_run(rt, v);
        if (v >= nown || v != (int)threadIdx.x) cur = rec[rt.start[r] + (v - rt.pre[r])];
        const int shp = rt.shift[r], exp_ = rt.ext[r];
        const R tt[3] = {cur.x, cur.y, cur.z};
        int dd[3];
        R w[3][P], unused[P];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int s;
            R f;
            decode_local<R>(tt[d], (exp_ >> (8 * d)) & 255, s, f);
            if constexpr (sizeof(R) == 4 && !TAB) {
                // mixed form: the polynomials in FP64, each weight rounded
                // once to FP32 (the FP32 evaluation carries a systematic
                // error of its rounded coefficients into every charge's
                // mesh cloud alike; FP64 FMAs issue at the FP32 rate here)
                double wd[P], ud[P];
                bspline<P, double, false>((double)f, wd, ud);
#pragma unroll
                for (int j = 0; j < P; ++j) w[d][j] = (R)wd[j];
            } else {
                stencil_weights<P, R, false, TAB>(f, g, w[d], unused);
            }
            // tile coordinate of the stencil start: negative for a charge of
            // the lower neighbour
            dd[d] = s + ((shp >> (8 * d)) & 255) - 128;
        }
        unsigned vy = 0, vz = 0;
#pragma unroll
        for (int j = 0; j < P; ++j) {
            vy |= ((unsigned)(dd[1] + j) < (unsigned)lim_y) ? (1u << j) : 0u;
            vz |= ((unsigned)(dd[2] + j) < (unsigned)lim_z) ? (1u << j) : 0u;
        }
        // charge and fixed-point scale folded into the z and x coefficients
        const R qv = cur.w;
#pragma unroll
        for (int j = 0; j < P; ++j) {
            w[2][j] *= qv;
            w[0][j] *= scale;
        }
        // first point of the stencil (24-bit products: |dd| < 2^7, plane <
        // 2^16); only valid rows and planes are touched.  A row's address is
        // this lane's first point plus a wave-uniform offset (scalar
        // arithmetic), one vector add per row.
        AC* const p0 = acc + (__mul24(dd[2], plane) + __mul24(dd[1], pitch) + (dd[0] + H));
        // dither of the plane's first point (mixed form; unused in FP64)
        float dz = dither_seed(cur);
        // z planes in a rolled loop; the plane's z weight is element 0 of
        // the register array, shifted down one per plane
#pragma unroll 1
        for (int jz = 0; jz < P; ++jz) {
            if (vz & 1u) {
                const R wz = w[2][0];
                const int zoff = __builtin_amdgcn_readfirstlane(jz * plane);
#pragma unroll
                for (int jy = 0; jy < P; ++jy) {
                    if (vy >> jy & 1u) {
                        const R wzy = wz * w[1][jy];
                        AC* row = p0 + __builtin_amdgcn_readfirstlane(zoff + jy * pitch);
                        // dz is in [0, 1) already: the first row takes it as it is
                        const float dy = jy == 0 ? dz : fract1(dz + (float)jy * DITHER_Y);
#pragma unroll
                        for (int jx = 0; jx < P; ++jx) Acc<AC>::add(row + jx, wzy, w[0][jx], dy);
                    }
                }
            }
            vz >>= 1;
            dz = fract1(dz + DITHER_Z);
#pragma unroll
            for (int j = 0; j < P - 1; ++j) w[2][j] = w[2][j + 1];
        }
    }
    __syncthreads();

    // periodic fold of single-tile axes: points K .. K + H - 1 onto 0 .. H - 1
    if (g.ntile[0] == 1) {
        const int rows = a.rows_y * a.planes_z;
        for (int i = threadIdx.x; i < rows * H; i += blockDim.x) {
            AC* row = acc + (i / H) * pitch + H;
            const int x = i % H;
            row[x] += row[g.K[0] + x];
        }
        __syncthreads();
    }
    if (g.ntile[1] == 1) {
        const int n = ext[0] * H * a.planes_z;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const int x = i % ext[0], y = (i / ext[0]) % H, z = i / (ext[0] * H);
            AC* p = acc + z * plane + H + x;
            p[y * pitch] += p[(g.K[1] + y) * pitch];
        }
        __syncthreads();
    }
    if (g.ntile[2] == 1) {
        const int n = ext[0] * ext[1] * H;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const int x = i % ext[0], y = (i / ext[0]) % ext[1], z = i / (ext[0] * ext[1]);
            AC* p = acc + y * pitch + H + x;
            p[z * plane] += p[(g.K[2] + z) * plane];
        }
        __syncthreads();
    }

    // flush: every point of the tile is owned here; coalesced stores.  The
    // thread's points are i = threadIdx.x + k blockDim.x in x-fastest order;
    // their coordinates advance by carries instead of a division per point
    // (integer division by a runtime value is a long instruction sequence).
    const int ex = ext[0], ey = ext[1], ez = ext[2];
    const double unit = ldexp(1.0, -e);
    const int bq = (int)blockDim.x / ex, bx = (int)blockDim.x - bq * ex;  // step in rows and in x
    const int by = bq % ey, bz = bq / ey;
    int lx = (int)threadIdx.x % ex, q = (int)threadIdx.x / ex;
    int ly = q % ey, lz = q / ey;
    while (lz < ez) {
        const double v = (double)acc[lz * plane + ly * pitch + H + lx] * unit;
        const size_t gidx = ((size_t)(T0[2] + lz) * g.K[1] + (T0[1] + ly)) * g.K[0] + (T0[0] + lx);
        ((R*)a.rho)[gidx] = (R)v;
        if (a.rho_user) a.rho_user[gidx] = v;
        lx += bx;
        const int cx = lx >= ex ? 1 : 0;
        lx -= cx * ex;
        ly += by + cx;
        const int cy = ly >= ey ? 1 : 0;
        ly -= cy * ey;
        lz += bz + cy;
    }
}

template <int P, typename R, typename A, bool TAB>
__device__ __forceinline__ void spread_kernel(const SpreadArgs& a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ RunTable rt;
    __shared__ int wmax[16];
    const MapGeo& g = a.g;

    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    int t[3];
    tile_coords(g, tile, t);
    const int T0[3] = {t[0] * g.B[0], t[1] * g.B[1], t[2] * g.B[2]};
    const int ext[3] = {tile_extent(g, 0, t[0]), tile_extent(g, 1, t[1]), tile_extent(g, 2, t[2])};

    // The thread's first visit is an own charge whenever the tile has enough
    // of them; its record is loaded before the accumulator is cleared.
    using RT = typename Rec<R>::T;
    const RT* __restrict__ rec = (const RT*)a.rec;
    const int own0 = a.offsets[tile * NCLASS * g.bin_stride], own1 = a.offsets[(tile + 1) * NCLASS * g.bin_stride];
    RT cur{};
    if (own0 + (int)threadIdx.x < own1) cur = rec[own0 + threadIdx.x];

    // Accumulator layout: rows of pitch_x points hold x in [-H, B_x + H)
    // (x index + H); rows_y rows per plane, planes_z planes.  The x margins
    // take the parts of stencils that fall outside the tile along x, so the
    // x loop needs no test; along y and z out-of-tile points are skipped.  On
    // an axis that is a single tile, stencils wrap: the points past K land in
    // margin rows / planes (y, z) or the right x margin and are folded back
    // onto the start of the axis before the flush.  The LDS holds 8 bytes per
    // point (a 32-bit tile uses the first half), then the occupancy count.
    long long* acc8 = (long long*)smem_raw;
    int* occ = (int*)(smem_raw + a.occ_off);
    const int nacc = a.pitch_x * a.rows_y * a.planes_z;
    const int nocc = a.occ_n[0] * a.occ_n[1] * a.occ_n[2];
    for (int i = threadIdx.x; i < nacc; i += blockDim.x) acc8[i] = 0;
    for (int i = threadIdx.x; i < nocc; i += blockDim.x) occ[i] = 0;
    build_run_table(g, t, a.offsets, rt);
    __syncthreads();
    const int total = rt.pre[NRUNS];
    const double qmax = a.stats[1];
    const int nown = own1 - own0;
    if (sizeof(A) == 8) {
        spread_tile<P, R, long long, TAB>(a, rt, acc8, fixed_point_exponent<P, 64>(total, qmax), cur, nown, T0, ext);
    } else if (total > WIDE_VISITS || wide_charge_range(a)) {
        spread_tile<P, R, long long, TAB>(a, rt, acc8, contribution_exponent<P>(qmax), cur, nown, T0, ext);
    } else {
        const int reach = count_pass(a, rt, occ, wmax, cur, nown, ext);
        if (reach > WIDE_REACH)
            spread_tile<P, R, long long, TAB>(a, rt, acc8, contribution_exponent<P>(qmax), cur, nown, T0, ext);
        else
            spread_tile<P, R, int, TAB>(a, rt, (int*)smem_raw, fixed_point_exponent<P, 32>(reach, qmax), cur, nown,
                                        T0, ext);
    }
}

// ---- push form (mixed precision) ------------------------------------------
// Each workgroup sums the whole stencils of its own tile's charges into an
// LDS box of (B_x + H) x (B_y + H) x (B_z + H) points, H = P - 1: the tile
// plus the H points past its upper faces that those stencils reach.  No
// charge is read by another tile and no row is clipped, so every issued LDS
// atomic lane is live (the owner-computes form above pulls the lower
// neighbours' charges and clips their stencils to the tile, which leaves
// about half the atomic lanes idle).  The box is flushed as FP32 partial
// sums; k_fold then adds, for each mesh point, the boxes of the (up to 8)
// tiles whose boxes hold it, in a fixed order.  The sums in LDS are the same
// exact fixed-point sums with the same dithered rounding; the exponent is
// set from the occupancy count of the tile's own charges.

// Occupancy count of the tile's own charges (stencil starts in [0, ext)),
// then the reach bound over the box (reach_bound's windows at the occupied
// cells bound every box point: a point past the tile is reached by a subset
// of the starts that reach the tile's last points).  Ends synchronised.
__device__ __forceinline__ int count_pass_own(const SpreadArgs& a, const float4* __restrict__ rec, int own0,
                                              int nown, int* occ, int* wmax, float4 cur, const int (&ext)[3])
{
    for (int v = threadIdx.x; v < nown; v += blockDim.x) {
        if (v != (int)threadIdx.x) cur = rec[own0 + v];
        const float tt[3] = {cur.x, cur.y, cur.z};
        int dd[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            float f;
            decode_local<float>(tt[d], ext[d], dd[d], f);
        }
        atomicAdd(&occ[occ_cell(a, dd)], 1);
    }
    __syncthreads();
    reach_bound(a, occ, ext, wmax);
    __syncthreads();
    int reach = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) reach = max(reach, wmax[w]);
    return reach;
}

template <int P, typename AC, bool TAB>
__device__ __forceinline__ void push_tile(const SpreadArgs& a, AC* acc, int e, float4 cur, int own0, int nown,
                                          const int (&ext)[3], float* __restrict__ out)
{
    const MapGeo& g = a.g;
    const float4* __restrict__ rec = (const float4*)a.rec;
    const int pitch = a.box_pitch;
    const int plane = pitch * a.box_rows;
    const float scale = (float)ldexp(1.0, e);
    for (int v = threadIdx.x; v < nown; v += blockDim.x) {
        if (v != (int)threadIdx.x) cur = rec[own0 + v];
        const float tt[3] = {cur.x, cur.y, cur.z};
        int sl[3];
        float w[3][P], unused[P];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            float f;
            decode_local<float>(tt[d], ext[d], sl[d], f);
            if constexpr (!TAB) {
                // the polynomials in FP64, each weight rounded once to FP32
                double wd[P], ud[P];
                bspline<P, double, false>((double)f, wd, ud);
#pragma unroll
                for (int j = 0; j < P; ++j) w[d][j] = (float)wd[j];
            } else {
                stencil_weights<P, float, false, TAB>(f, g, w[d], unused);
            }
        }
#pragma unroll
        for (int j = 0; j < P; ++j) {
            w[2][j] *= cur.w;
            w[0][j] *= scale;
        }
        // the stencil's first point (box coordinates = tile coordinates);
        // rows and planes add wave-uniform offsets
        AC* const p0 = acc + (__mul24(sl[2], plane) + __mul24(sl[1], pitch) + sl[0]);
        float dz = dither_seed(cur);
#pragma unroll 1
        for (int jz = 0; jz < P; ++jz) {
            const float wz = w[2][0];
            const int zoff = __builtin_amdgcn_readfirstlane(jz * plane);
#pragma unroll
            for (int jy = 0; jy < P; ++jy) {
                const float wzy = wz * w[1][jy];
                AC* row = p0 + __builtin_amdgcn_readfirstlane(zoff + jy * pitch);
                const float dy = jy == 0 ? dz : fract1(dz + (float)jy * DITHER_Y);
#pragma unroll
                for (int jx = 0; jx < P; ++jx) Acc<AC>::add(row + jx, wzy, w[0][jx], dy);
            }
            dz = fract1(dz + DITHER_Z);
#pragma unroll
            for (int j = 0; j < P - 1; ++j) w[2][j] = w[2][j + 1];
        }
    }
    __syncthreads();
    // flush the whole box (points past a ragged tile's box hold zero)
    const double unit = ldexp(1.0, -e);
    const int nbox = plane * a.box_planes;
    for (int i = threadIdx.x; i < nbox; i += blockDim.x) out[i] = (float)((double)acc[i] * unit);
}

template <int P, bool TAB>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void k_spread_push(SpreadArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int wmax[16];
    const MapGeo& g = a.g;
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    int t[3];
    tile_coords(g, tile, t);
    const int ext[3] = {tile_extent(g, 0, t[0]), tile_extent(g, 1, t[1]), tile_extent(g, 2, t[2])};
    const float4* __restrict__ rec = (const float4*)a.rec;
    const int own0 = a.offsets[tile * NCLASS * g.bin_stride], own1 = a.offsets[(tile + 1) * NCLASS * g.bin_stride];
    const int nown = own1 - own0;
    float4 cur{};
    if ((int)threadIdx.x < nown) cur = rec[own0 + threadIdx.x];
    // LDS: the box, 8 bytes per point (a 32-bit tile uses the first half),
    // then the occupancy count
    long long* acc8 = (long long*)smem_raw;
    int* occ = (int*)(smem_raw + a.occ_off);
    const int nocc = a.occ_n[0] * a.occ_n[1] * a.occ_n[2];
    // a 32-bit tile clears the first half only
    const bool wide = nown > WIDE_VISITS || wide_charge_range(a);
    const int nclear = wide ? a.box_stride : (a.box_stride + 1) / 2;
    for (int i = threadIdx.x; i < nclear; i += blockDim.x) acc8[i] = 0;
    for (int i = threadIdx.x; i < nocc; i += blockDim.x) occ[i] = 0;
    __syncthreads();
    float* out = a.box + (size_t)tile * a.box_stride;
    const double qmax = a.stats[1];
    if (wide) {
        push_tile<P, long long, TAB>(a, acc8, contribution_exponent<P>(qmax), cur, own0, nown, ext, out);
    } else {
        const int reach = count_pass_own(a, rec, own0, nown, occ, wmax, cur, ext);
        if (reach > WIDE_REACH) {
            // 64-bit sums after all: clear the second half of the box too
            for (int i = (a.box_stride + 1) / 2 + (int)threadIdx.x; i < a.box_stride; i += blockDim.x) acc8[i] = 0;
            __syncthreads();
            push_tile<P, long long, TAB>(a, acc8, contribution_exponent<P>(qmax), cur, own0, nown, ext, out);
        } else {
            push_tile<P, int, TAB>(a, (int*)smem_raw, fixed_point_exponent<P, 32>(reach, qmax), cur, own0, nown,
                                   ext, out);
        }
    }
}

// Fold of the push form: point (lx, ly, lz) of a tile sums its own box
// value and, for each set of axes d along which l_d < H, the box value of
// the lower neighbour across those axes (periodic) at l_d + that
// neighbour's extent; the up-to-8 terms are added
// in FP64 in a fixed order (own tile first, then the neighbours by mask).
// The own values and the written rows of the mesh are coalesced.
struct FoldArgs {
    const float* box;
    float* rho;          // plan mesh (FFT input), FP32
    double* rho_user;    // caller's FP64 mesh or null
    MapGeo g;
    int pitch, rows, stride;
};

constexpr int FOLD_THREADS = 256;

// Workgroup (bx, FOLD_THREADS / bx): x of the tile along threadIdx.x (bx =
// B_x rounded up to 32, at most 64), rows (y, z) of the tile along
// threadIdx.y and blockIdx.y; the tile's geometry is uniform per workgroup.
__global__ __launch_bounds__(FOLD_THREADS) void k_fold(FoldArgs f)
{
    const MapGeo& g = f.g;
    const int H = g.halo;
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    int t[3];
    tile_coords(g, tile, t);
    const int ext[3] = {tile_extent(g, 0, t[0]), tile_extent(g, 1, t[1]), tile_extent(g, 2, t[2])};
    const int lx = threadIdx.x;
    const int r = (int)(blockIdx.y * blockDim.y + threadIdx.y);
    if (lx >= ext[0] || r >= ext[1] * ext[2]) return;
    const int lz = r / ext[1], ly = r - lz * ext[1];
    // lower neighbours (periodic) and their extents
    int tl[3], el[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        tl[d] = t[d] == 0 ? g.ntile[d] - 1 : t[d] - 1;
        el[d] = tile_extent(g, d, tl[d]);
    }
    const int mask = (lx < H ? 1 : 0) | (ly < H ? 2 : 0) | (lz < H ? 4 : 0);
    // The terms any lane of the wavefront needs (a uniform mask) are loaded
    // first, all in flight together, then added in the fixed order; a lane
    // that needs fewer terms reads its own point for the others and drops
    // them.  (Loading and adding term by term waits out one memory round
    // trip per term.)
    const int wmask = (__any(mask & 1) ? 1 : 0) | (__any(mask & 2) ? 2 : 0) | (__any(mask & 4) ? 4 : 0);
    const size_t own = (size_t)tile * f.stride + (size_t)(lz * f.rows + ly) * f.pitch + lx;
    float v[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        v[m] = 0.0f;
        if ((m & wmask) != m) continue;
        size_t idx = own;
        if ((m & mask) == m) {
            const int sx = (m & 1) ? tl[0] : t[0], sy = (m & 2) ? tl[1] : t[1], sz = (m & 4) ? tl[2] : t[2];
            const int cx = lx + ((m & 1) ? el[0] : 0), cy = ly + ((m & 2) ? el[1] : 0),
                      cz = lz + ((m & 4) ? el[2] : 0);
            idx = (size_t)((sz * g.ntile[1] + sy) * g.ntile[0] + sx) * f.stride + (size_t)(cz * f.rows + cy) * f.pitch + cx;
        }
        v[m] = f.box[idx];
    }
    double sum = 0.0;
#pragma unroll
    for (int m = 0; m < 8; ++m)
        if ((m & mask) == m) sum += (double)v[m];
    const size_t gi = ((size_t)(t[2] * g.B[2] + lz) * g.K[1] + (t[1] * g.B[1] + ly)) * g.K[0] + (t[0] * g.B[0] + lx);
    f.rho[gi] = (float)sum;
    if (f.rho_user) f.rho_user[gi] = sum;
}

template <bool TAB>
hipError_t dispatch_push(int P, dim3 grid, dim3 block, size_t lds, hipStream_t st, const SpreadArgs& a)
{
    switch (P) {
    case 2: k_spread_push<2, TAB><<<grid, block, lds, st>>>(a); break;
    case 3: k_spread_push<3, TAB><<<grid, block, lds, st>>>(a); break;
    case 4: k_spread_push<4, TAB><<<grid, block, lds, st>>>(a); break;
    case 5: k_spread_push<5, TAB><<<grid, block, lds, st>>>(a); break;
    case 6: k_spread_push<6, TAB><<<grid, block, lds, st>>>(a); break;
    case 7: k_spread_push<7, TAB><<<grid, block, lds, st>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// The mixed form asks for eight wavefronts per SIMD (two 1024-thread
// workgroups per CU), which its register use allows without spilling; the
// FP64 form needs more registers and runs with fewer.
template <int P, bool TAB>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void k_spread(SpreadArgs a)
{
    spread_kernel<P, float, int, TAB>(a);
}
template <int P, bool TAB>
__global__ __launch_bounds__(1024) void k_spread64(SpreadArgs a)
{
    spread_kernel<P, double, long long, TAB>(a);
}

template <int P, bool TAB>
void launch_spread_p(bool mixed, dim3 grid, dim3 block, size_t lds, hipStream_t st, const SpreadArgs& a)
{
    if (mixed)
        k_spread<P, TAB><<<grid, block, lds, st>>>(a);
    else
        k_spread64<P, TAB><<<grid, block, lds, st>>>(a);
}

template <bool TAB>
hipError_t dispatch_spread(bool mixed, int P, dim3 grid, dim3 block, size_t lds, hipStream_t st, const SpreadArgs& a)
{
    switch (P) {
    case 2: launch_spread_p<2, TAB>(mixed, grid, block, lds, st, a); break;
    case 3: launch_spread_p<3, TAB>(mixed, grid, block, lds, st, a); break;
    case 4: launch_spread_p<4, TAB>(mixed, grid, block, lds, st, a); break;
    case 5: launch_spread_p<5, TAB>(mixed, grid, block, lds, st, a); break;
    case 6: launch_spread_p<6, TAB>(mixed, grid, block, lds, st, a); break;
    case 7: launch_spread_p<7, TAB>(mixed, grid, block, lds, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

namespace {

// Coarse cells of the occupancy count per axis: starts lie in [-H, B), so
// B + H of them, in cells of a power-of-two edge of at least 4 points and at
// most 16 cells; an axis that is a single tile is one cell (its stencils
// wrap onto the tile).
struct OccGeo {
    int shift[3], n[3], k[3];
};
OccGeo occ_geo(const MapGeo& g)
{
    OccGeo o{};
    for (int d = 0; d < 3; ++d) {
        const int span = g.B[d] + g.halo;
        if (g.ntile[d] == 1) {
            o.shift[d] = 30;
            o.n[d] = 1;
            o.k[d] = 0;
        } else {
            int sh = 2;
            while ((span + (1 << sh) - 1) >> sh > 16) ++sh;
            o.shift[d] = sh;
            o.n[d] = (span + (1 << sh) - 1) >> sh;
            o.k[d] = (g.halo + (1 << sh) - 1) >> sh;
        }
    }
    return o;
}

int spread_rows(const MapGeo& g, int d) { return g.B[d] + (g.ntile[d] == 1 ? g.halo : 0); }

size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }

// LDS of k_spread: the accumulator (8 bytes per point in both forms, see
// k_spread), then the occupancy count; the count's offset and the total.
struct SpreadLds {
    size_t occ_off, total;
};
SpreadLds spread_lds_layout(const MapGeo& g)
{
    const OccGeo o = occ_geo(g);
    const size_t nacc = (size_t)(g.B[0] + 2 * g.halo) * spread_rows(g, 1) * spread_rows(g, 2);
    SpreadLds l{};
    l.occ_off = align16(nacc * sizeof(long long));
    l.total = l.occ_off + align16((size_t)o.n[0] * o.n[1] * o.n[2] * sizeof(int));
    return l;
}

}  // namespace

size_t spread_lds_bytes(const MapGeo& g) { return spread_lds_layout(g).total; }

// Points of one tile's box in the push form: (B_x + H)(B_y + H)(B_z + H).
int64_t spread_box_points(const MapGeo& g)
{
    return (int64_t)(g.B[0] + g.halo) * (g.B[1] + g.halo) * (g.B[2] + g.halo);
}

// LDS of k_spread_push: the box at 8 bytes per point, then the occupancy
// count.
SpreadLds push_lds_layout(const MapGeo& g)
{
    const OccGeo o = occ_geo(g);
    SpreadLds l{};
    l.occ_off = align16((size_t)spread_box_points(g) * sizeof(long long));
    l.total = l.occ_off + align16((size_t)o.n[0] * o.n[1] * o.n[2] * sizeof(int));
    return l;
}
size_t spread_push_lds_bytes(const MapGeo& g) { return push_lds_layout(g).total; }

hipError_t launch_spread(pppm_plan_s* pl, double* rho_user)
{
    if (pl->spread_push) {
        const MapGeo& g = pl->geo;
        SpreadArgs a{};
        a.g = g;
        a.offsets = pl->offsets;
        a.rec = pl->records;
        a.stats = pl->eterms + 6;
        a.box = pl->box;
        a.box_pitch = g.B[0] + g.halo;
        a.box_rows = g.B[1] + g.halo;
        a.box_planes = g.B[2] + g.halo;
        a.box_stride = (int)spread_box_points(g);
        const OccGeo o = occ_geo(g);
        const SpreadLds l = push_lds_layout(g);
        a.occ_off = (int)l.occ_off;
        for (int d = 0; d < 3; ++d) {
            a.occ_shift[d] = o.shift[d];
            a.occ_n[d] = o.n[d];
            a.occ_k[d] = o.k[d];
        }
        dim3 grid(g.ntiles), block(pl->spread_cfg.threads);
        const hipError_t e = g.wtab ? dispatch_push<true>(pl->p.order, grid, block, l.total, pl->stream, a)
                                    : dispatch_push<false>(pl->p.order, grid, block, l.total, pl->stream, a);
        if (e != hipSuccess) return e;
        FoldArgs f{};
        f.box = pl->box;
        f.rho = (float*)pl->rho;
        f.rho_user = rho_user;
        f.g = g;
        f.pitch = a.box_pitch;
        f.rows = a.box_rows;
        f.stride = a.box_stride;
        const int bx = g.B[0] <= 32 ? 32 : 64;
        const int by = FOLD_THREADS / bx;
        const int rows = g.B[1] * g.B[2];
        k_fold<<<dim3(g.ntiles, (rows + by - 1) / by), dim3(bx, by), 0, pl->stream>>>(f);
        return hipGetLastError();
    }
    SpreadArgs a{};
    a.g = pl->geo;
    a.offsets = pl->offsets;
    a.rec = pl->records;
    a.rho = pl->rho;
    a.rho_user = rho_user;
    a.pitch_x = pl->geo.B[0] + 2 * pl->geo.halo;
    a.rows_y = spread_rows(pl->geo, 1);
    a.planes_z = spread_rows(pl->geo, 2);
    a.stats = pl->eterms + 6;
    const OccGeo o = occ_geo(pl->geo);
    const SpreadLds l = spread_lds_layout(pl->geo);
    a.occ_off = (int)l.occ_off;
    for (int d = 0; d < 3; ++d) {
        a.occ_shift[d] = o.shift[d];
        a.occ_n[d] = o.n[d];
        a.occ_k[d] = o.k[d];
    }
    const size_t lds = l.total;
    dim3 grid(pl->geo.ntiles), block(pl->spread_cfg.threads);
    const bool tab = pl->geo.wtab != nullptr;
    return tab ? dispatch_spread<true>(pl->mixed, pl->p.order, grid, block, lds, pl->stream, a)
               : dispatch_spread<false>(pl->mixed, pl->p.order, grid, block, lds, pl->stream, a);
}

}  // namespace pppm
