// make_rho: the paper's Map-Charge (Section 3.1).  Each charge adds
// q * wx * wy * wz to the P^3 mesh points of its stencil.
//
// GPU design (owner computes): one workgroup owns one tile of mesh points and
// accumulates it in LDS.  It reads every binned charge whose stencil reaches
// into the tile - the charges of the tile's own sub-bricks and those of the
// sub-bricks up to P - 1 points below it - and adds the part of each stencil
// that falls inside the tile with LDS atomics.  Every mesh point is owned by
// exactly one tile, so the tile is flushed to the global mesh with plain
// coalesced FP64 stores: no global atomics and no zero-fill of the mesh.
// This is the GPU counterpart of the paper's per-thread private grids
// ("rethread"): privatise, accumulate, then combine - here the combine is a
// disjoint ownership of the output.
#include "runs.h"

namespace pppm {

namespace {

struct SpreadArgs {
    TileGeo tg;
    const int* offsets;
    const void* rec;
    double* rho;
    double* rho_user;
    int pitch_x;  // LDS row pitch (points)
};

template <int P, typename R>
__global__ __launch_bounds__(512) void k_spread(SpreadArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int lists[3 * MAXL];
    __shared__ int cnts[3];
    __shared__ int scratch[17];
    const TileGeo& tg = a.tg;

    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int tix = tile % tg.ntile[0];
    const int tiy = (tile / tg.ntile[0]) % tg.ntile[1];
    const int tiz = tile / (tg.ntile[0] * tg.ntile[1]);
    const int T0[3] = {tix * tg.B[0], tiy * tg.B[1], tiz * tg.B[2]};
    const int ext[3] = {min(tg.B[0], tg.K[0] - T0[0]), min(tg.B[1], tg.K[1] - T0[1]),
                        min(tg.B[2], tg.K[2] - T0[2])};

    // LDS layout: accumulator tile, then the run table
    R* acc = (R*)smem_raw;
    const int plane = a.pitch_x * tg.B[1];
    const int nacc = plane * tg.B[2];
    int* run_start = (int*)(acc + nacc);
    int* run_sb = run_start + MAX_RUNS;
    int* prefix = run_sb + MAX_RUNS;

    for (int i = threadIdx.x; i < nacc; i += blockDim.x) acc[i] = R(0);
    const int nruns = build_runs(tg, T0, ext, P - 1, a.offsets, lists, cnts, run_start, prefix, run_sb, scratch);
    if (nruns < 0) return;
    const int total = prefix[nruns];

    using RT = typename Rec<R>::T;
    const RT* __restrict__ rec = (const RT*)a.rec;
    for (int v = threadIdx.x; v < total; v += blockDim.x) {
        const int r = find_run(prefix, nruns, v);
        const RT pr = rec[run_start[r] + (v - prefix[r])];
        const int sbp = run_sb[r];
        const int sbc[3] = {sbp & 1023, (sbp >> 10) & 1023, sbp >> 20};
        const R tt[3] = {pr.x, pr.y, pr.z};
        int l[3][P];
        unsigned valid[3];
        R w[3][P], unused[P];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int s;
            R f;
            decode_axis<R>(tt[d], sbc[d], tg.K[d], s, f);
            bspline<P, R, false>(f, w[d], unused);
            const int dd = s - T0[d];
            const int wrap = tg.K[d] - T0[d];
            unsigned m = 0;
#pragma unroll
            for (int j = 0; j < P; ++j) {
                int lj = dd + j;
                if (lj >= wrap) lj -= tg.K[d];
                l[d][j] = lj;
                m |= ((unsigned)lj < (unsigned)ext[d]) ? (1u << j) : 0u;
            }
            valid[d] = m;
        }
        const R qv = pr.w;
        // z planes in a rolled loop; the plane's z data is element 0 of the
        // register arrays, shifted down one per plane
        unsigned vz = valid[2];
#pragma unroll 1
        for (int jz = 0; jz < P; ++jz) {
            if (vz & 1u) {
                const R wz = qv * w[2][0];
                const int bz = l[2][0] * plane;
#pragma unroll
                for (int jy = 0; jy < P; ++jy) {
                    if (!(valid[1] >> jy & 1u)) continue;
                    const R wzy = wz * w[1][jy];
                    R* row = acc + bz + l[1][jy] * a.pitch_x;
#pragma unroll
                    for (int jx = 0; jx < P; ++jx) {
                        if (valid[0] >> jx & 1u) atomicAdd(row + l[0][jx], wzy * w[0][jx]);
                    }
                }
            }
            vz >>= 1;
#pragma unroll
            for (int j = 0; j < P - 1; ++j) {
                w[2][j] = w[2][j + 1];
                l[2][j] = l[2][j + 1];
            }
        }
    }
    __syncthreads();

    // flush: every point of the tile is owned here; coalesced FP64 stores
    const int ex = ext[0], ey = ext[1], ez = ext[2];
    const int npts = ex * ey * ez;
    for (int i = threadIdx.x; i < npts; i += blockDim.x) {
        const int lx = i % ex, ly = (i / ex) % ey, lz = i / (ex * ey);
        const double v = (double)acc[lz * plane + ly * a.pitch_x + lx];
        const size_t gidx = ((size_t)(T0[2] + lz) * tg.K[1] + (T0[1] + ly)) * tg.K[0] + (T0[0] + lx);
        a.rho[gidx] = v;
        if (a.rho_user) a.rho_user[gidx] = v;
    }
}

template <typename R>
hipError_t dispatch_spread(int P, dim3 grid, dim3 block, size_t lds, hipStream_t st, const SpreadArgs& a)
{
    switch (P) {
    case 2: k_spread<2, R><<<grid, block, lds, st>>>(a); break;
    case 3: k_spread<3, R><<<grid, block, lds, st>>>(a); break;
    case 4: k_spread<4, R><<<grid, block, lds, st>>>(a); break;
    case 5: k_spread<5, R><<<grid, block, lds, st>>>(a); break;
    case 6: k_spread<6, R><<<grid, block, lds, st>>>(a); break;
    case 7: k_spread<7, R><<<grid, block, lds, st>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

TileGeo make_tiles(const pppm_plan_s* pl, const LaunchCfg& c)
{
    TileGeo t{};
    for (int d = 0; d < 3; ++d) {
        t.K[d] = pl->geo.K[d];
        t.nsb[d] = pl->geo.nsb[d];
        t.B[d] = c.tile[d];
        t.ntile[d] = (t.K[d] + t.B[d] - 1) / t.B[d];
    }
    t.ntiles = t.ntile[0] * t.ntile[1] * t.ntile[2];
    return t;
}

static int spread_pitch(const LaunchCfg& c) { return c.tile[0] + 1; }

size_t spread_lds_bytes(const pppm_plan_s* pl, const LaunchCfg& c)
{
    const size_t nacc = (size_t)spread_pitch(c) * c.tile[1] * c.tile[2];
    return nacc * pl->rsize + 3 * MAX_RUNS * sizeof(int) + sizeof(int);
}

int runs_needed(const pppm_plan_s* pl, const LaunchCfg& c, bool spread)
{
    // worst case over tiles: own sub-bricks plus the halo ones, per axis
    long total = 1;
    const int halo = spread ? pl->p.order - 1 : 0;
    for (int d = 0; d < 3; ++d) {
        const int K = pl->geo.K[d];
        int n;
        if (c.tile[d] + halo >= K)
            n = pl->geo.nsb[d];
        else
            n = (c.tile[d] + halo + SB - 1) / SB + 1;
        if (n > MAXL) return 1 << 30;
        total *= n;
    }
    return (int)total;
}

hipError_t launch_spread(pppm_plan_s* pl, double* rho_user)
{
    const LaunchCfg& c = pl->spread_cfg;
    SpreadArgs a{};
    a.tg = make_tiles(pl, c);
    a.offsets = pl->offsets;
    a.rec = pl->records;
    a.rho = pl->rho;
    a.rho_user = rho_user;
    a.pitch_x = spread_pitch(c);
    const size_t lds = spread_lds_bytes(pl, c);
    dim3 grid(a.tg.ntiles), block(c.threads);
    if (pl->mixed) return dispatch_spread<float>(pl->p.order, grid, block, lds, pl->stream, a);
    return dispatch_spread<double>(pl->p.order, grid, block, lds, pl->stream, a);
}

}  // namespace pppm
