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
// disjoint ownership of the output.
//
// Accumulator.  On gfx950 the LDS float atomic add (ds_add_f32) is processed
// at about one lane every three clocks for any non-uniform address pattern,
// some 30x slower than the integer one (ds_add_u32).  The mixed-precision
// form therefore accumulates each tile in exact 32-bit fixed point: every
// FP32 contribution q wx wy wz is rounded to an integer multiple of 2^-e and
// added with ds_add_u32.  Integer addition is associative (modulo 2^32), so
// the sum is exact and independent of the order of the atomics, and it is
// correct whenever the final value fits, |rho_m| 2^e < 2^31.  e is chosen per
// tile from a bound on any of its points: each charge read by the tile adds
// at most max|q| wmax(P)^3 to a point, with one bit of headroom.  The flush
// converts each exact sum to FP64; that value goes to the caller's FP64 mesh
// when one is asked for, and, rounded to FP32, to the plan's FFT input (the
// mixed form transforms in FP32).  The FP64 form does the same in 64-bit
// fixed point (FP64 products rounded to integers, ds_add_u64, 2^62 bound):
// faster than ds_add_f64 and, like the mixed form, independent of the order
// of the atomics; it keeps an FP64 FFT input.
#include "tiles.h"

namespace pppm {

namespace {

struct SpreadArgs {
    MapGeo g;
    const int* offsets;
    const void* rec;
    void* rho;            // plan mesh of type R (the FFT input)
    double* rho_user;     // caller's FP64 mesh or null
    const double* stats;  // [1] max |q|
    int pitch_x;          // LDS row pitch (points): B_x + 2 (P - 1)
    int rows_y;           // LDS rows per plane: B_y, + P - 1 on a single-tile axis
    int planes_z;         // LDS planes: B_z, + P - 1 on a single-tile axis
};

// Largest value of the order-P B-spline (P = 2..7), rounded up.
__host__ __device__ constexpr double bspline_max(int P)
{
    return P == 2 ? 1.0 : P == 3 ? 0.7501 : P == 4 ? 0.6668 : P == 5 ? 0.5991 : P == 6 ? 0.5501 : 0.5111;
}

// Fixed-point exponent of a tile reading `visits` charges (see above) for a
// BITS-bit accumulator: the bound times 2^e stays below 2^(BITS - 2), one bit
// of headroom.
template <int P, int BITS>
__device__ __forceinline__ int fixed_point_exponent(int visits, double qmax)
{
    const double wm = bspline_max(P);
    const double bound = (double)visits * qmax * wm * wm * wm;
    if (!(bound > 0.0)) return BITS - 2;
    int e = (int)floor(log2(ldexp(1.0, BITS - 2) / bound));
    return e < -60 ? -60 : (e > 120 ? 120 : e);
}

template <typename A> struct Acc;
template <> struct Acc<int> {
    // round half up, floor(v + 1/2), in one instruction (v_cvt_rpi_i32_f32)
    __device__ static void add(int* p, float v)
    {
        int r;
        asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(v));
        atomicAdd(p, r);
    }
};
template <> struct Acc<long long> {
    // FP64 form: 64-bit fixed point, the product rounded to nearest
    __device__ static void add(long long* p, double v)
    {
        atomicAdd((unsigned long long*)p, (unsigned long long)__double2ll_rn(v));
    }
};

template <int P, typename R, typename A, bool TAB>
__global__ __launch_bounds__(1024) void k_spread(SpreadArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ RunTable rt;
    const MapGeo& g = a.g;
    constexpr int H = P - 1;  // halo / margin width

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
    // onto the start of the axis before the flush.
    A* acc = (A*)smem_raw;
    const int pitch = a.pitch_x;
    const int plane = pitch * a.rows_y;
    const int nacc = plane * a.planes_z;
    for (int i = threadIdx.x; i < nacc; i += blockDim.x) acc[i] = A(0);
    build_run_table(g, t, a.offsets, rt);
    __syncthreads();
    const int total = rt.pre[NRUNS];
    int e = 0;
    if (sizeof(A) == 4) e = fixed_point_exponent<P, 32>(total, a.stats[1]);
    else e = fixed_point_exponent<P, 64>(total, a.stats[1]);
    const R scale = (R)ldexp(1.0, e);
    // valid y rows / z planes: [0, lim)
    const int lim_y = g.ntile[1] == 1 ? g.K[1] + H : ext[1];
    const int lim_z = g.ntile[2] == 1 ? g.K[2] + H : ext[2];

    for (int v = threadIdx.x; v < total; v += blockDim.x) {
        const int r = find_run(rt, v);
        if (v >= own1 - own0 || v != (int)threadIdx.x) cur = rec[rt.start[r] + (v - rt.pre[r])];
        const int shp = rt.shift[r], exp_ = rt.ext[r];
        const R tt[3] = {cur.x, cur.y, cur.z};
        int dd[3];
        R w[3][P], unused[P];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int s;
            R f;
            decode_local<R>(tt[d], (exp_ >> (8 * d)) & 255, s, f);
            stencil_weights<P, R, false, TAB>(f, g, w[d], unused);
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
        // first point of the stencil; only valid rows and planes are touched
        A* pz = acc + dd[2] * plane + dd[1] * pitch + (dd[0] + H);
        // z planes in a rolled loop; the plane's z weight is element 0 of
        // the register array, shifted down one per plane
#pragma unroll 1
        for (int jz = 0; jz < P; ++jz) {
            if (vz & 1u) {
                const R wz = w[2][0];
#pragma unroll
                for (int jy = 0; jy < P; ++jy) {
                    if (vy >> jy & 1u) {
                        const R wzy = wz * w[1][jy];
                        A* row = pz + jy * pitch;
#pragma unroll
                        for (int jx = 0; jx < P; ++jx) Acc<A>::add(row + jx, wzy * w[0][jx]);
                    }
                }
            }
            vz >>= 1;
            pz += plane;
#pragma unroll
            for (int j = 0; j < P - 1; ++j) w[2][j] = w[2][j + 1];
        }
    }
    __syncthreads();

    // periodic fold of single-tile axes: points K .. K + H - 1 onto 0 .. H - 1
    if (g.ntile[0] == 1) {
        const int rows = a.rows_y * a.planes_z;
        for (int i = threadIdx.x; i < rows * H; i += blockDim.x) {
            A* row = acc + (i / H) * pitch + H;
            const int x = i % H;
            row[x] += row[g.K[0] + x];
        }
        __syncthreads();
    }
    if (g.ntile[1] == 1) {
        const int n = ext[0] * H * a.planes_z;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const int x = i % ext[0], y = (i / ext[0]) % H, z = i / (ext[0] * H);
            A* p = acc + z * plane + H + x;
            p[y * pitch] += p[(g.K[1] + y) * pitch];
        }
        __syncthreads();
    }
    if (g.ntile[2] == 1) {
        const int n = ext[0] * ext[1] * H;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const int x = i % ext[0], y = (i / ext[0]) % ext[1], z = i / (ext[0] * ext[1]);
            A* p = acc + y * pitch + H + x;
            p[z * plane] += p[(g.K[2] + z) * plane];
        }
        __syncthreads();
    }

    // flush: every point of the tile is owned here; coalesced stores
    const int ex = ext[0], ey = ext[1], ez = ext[2];
    const int npts = ex * ey * ez;
    for (int i = threadIdx.x; i < npts; i += blockDim.x) {
        const int lx = i % ex, ly = (i / ex) % ey, lz = i / (ex * ey);
        const double v = ldexp((double)acc[lz * plane + ly * pitch + H + lx], -e);
        const size_t gidx = ((size_t)(T0[2] + lz) * g.K[1] + (T0[1] + ly)) * g.K[0] + (T0[0] + lx);
        ((R*)a.rho)[gidx] = (R)v;
        if (a.rho_user) a.rho_user[gidx] = v;
    }
}

template <typename R, typename A, bool TAB>
hipError_t dispatch_spread(int P, dim3 grid, dim3 block, size_t lds, hipStream_t st, const SpreadArgs& a)
{
    switch (P) {
    case 2: k_spread<2, R, A, TAB><<<grid, block, lds, st>>>(a); break;
    case 3: k_spread<3, R, A, TAB><<<grid, block, lds, st>>>(a); break;
    case 4: k_spread<4, R, A, TAB><<<grid, block, lds, st>>>(a); break;
    case 5: k_spread<5, R, A, TAB><<<grid, block, lds, st>>>(a); break;
    case 6: k_spread<6, R, A, TAB><<<grid, block, lds, st>>>(a); break;
    case 7: k_spread<7, R, A, TAB><<<grid, block, lds, st>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

namespace {
int spread_rows(const MapGeo& g, int d) { return g.B[d] + (g.ntile[d] == 1 ? g.halo : 0); }
}  // namespace

size_t spread_lds_bytes(const MapGeo& g, size_t acc_bytes)
{
    return (size_t)(g.B[0] + 2 * g.halo) * spread_rows(g, 1) * spread_rows(g, 2) * acc_bytes;
}

hipError_t launch_spread(pppm_plan_s* pl, double* rho_user)
{
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
    const size_t lds = spread_lds_bytes(pl->geo, pl->rsize);
    dim3 grid(pl->geo.ntiles), block(pl->spread_cfg.threads);
    const bool tab = pl->geo.wtab != nullptr;
    if (pl->mixed)
        return tab ? dispatch_spread<float, int, true>(pl->p.order, grid, block, lds, pl->stream, a)
                   : dispatch_spread<float, int, false>(pl->p.order, grid, block, lds, pl->stream, a);
    return tab ? dispatch_spread<double, long long, true>(pl->p.order, grid, block, lds, pl->stream, a)
               : dispatch_spread<double, long long, false>(pl->p.order, grid, block, lds, pl->stream, a);
}

}  // namespace pppm
