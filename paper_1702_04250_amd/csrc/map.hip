// Particle map (the per-atom part of the mapping functions, paper Section
// 3.1): wrap each charge into the box, find its stencil start and fraction,
// and counting-sort the charges by (tile, halo class) bin.  Three passes:
// count (with per-bin rank), scan, scatter into binned order.
#include "tiles.h"

namespace pppm {

namespace {

// Bin of a charge with stencil start s (wrapped into [0, K)); sl receives the
// start within the tile.
__device__ __forceinline__ int bin_of(const MapGeo& g, const int (&s)[3], int (&sl)[3])
{
    int t[3], cls = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        t[d] = s[d] / g.B[d];
        sl[d] = s[d] - t[d] * g.B[d];
        const int ext = tile_extent(g, d, t[d]);
        if (g.ntile[d] >= 2 && sl[d] >= ext - g.halo) cls |= 1 << d;
    }
    const int tile = (t[2] * g.ntile[1] + t[1]) * g.ntile[0] + t[0];
    return tile * NCLASS + class_pos(cls);
}

template <typename TI>
__global__ __launch_bounds__(MAP_THREADS) void k_map_count(int n, const TI* __restrict__ pos,
                                                            const TI* __restrict__ q, MapGeo g,
                                                            int* __restrict__ count,
                                                            int* __restrict__ slot,
                                                            double* __restrict__ qpart,
                                                            int* __restrict__ flags)
{
    __shared__ double red[3][MAP_THREADS / 64];
    const int i = blockIdx.x * MAP_THREADS + threadIdx.x;
    double qi = 0.0;
    if (i < n) {
        int s[3];
        double f[3];
        bool ok = true;
#pragma unroll
        for (int d = 0; d < 3; ++d)
            ok &= map_coord((double)pos[3 * (size_t)i + d], g.lo[d], g.h[d], g.K[d], g.shift, s[d], f[d]);
        qi = (double)q[i];
        if (!isfinite(qi)) ok = false;
        if (!ok && g.check_finite) atomicOr(flags, 1);
        int sl[3];
        slot[i] = atomicAdd(&count[bin_of(g, s, sl) * NSUB + (i & (NSUB - 1))], 1);
    }
    // charge sums for the self and background energy terms, and max |q|
    // (which bounds the mesh charge for the fixed-point spread)
    double a = qi, b = qi * qi, c = fabs(qi);
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        a += __shfl_down(a, d, 64);
        b += __shfl_down(b, d, 64);
        c = fmax(c, __shfl_down(c, d, 64));
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wid] = a;
        red[1][wid] = b;
        red[2][wid] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0, sc = 0.0;
        for (int w = 0; w < MAP_THREADS / 64; ++w) {
            sa += red[0][w];
            sb += red[1][w];
            sc = fmax(sc, red[2][w]);
        }
        qpart[3 * blockIdx.x] = sa;
        qpart[3 * blockIdx.x + 1] = sb;
        qpart[3 * blockIdx.x + 2] = sc;
    }
}

// Sum (part[b]) and maximum (part[nblocks + b]) of each SCAN_BLOCK-long chunk
// of the bin counts.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(int nbins_, int nblocks, const int* __restrict__ count,
                                                               int* __restrict__ part)
{
    __shared__ int scratch[17];
    __shared__ int wmax[SCAN_THREADS / 64];
    const int base = blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_ITEMS;
    int v = 0, m = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k)
        if (base + k < nbins_) {
            const int c = count[base + k];
            v += c;
            m = max(m, c);
        }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) m = max(m, __shfl_down(m, d, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    int total;
    block_exclusive_scan(v, scratch, &total);
    if (threadIdx.x == 0) {
        int mm = 0;
        for (int w = 0; w < SCAN_THREADS / 64; ++w) mm = max(mm, wmax[w]);
        part[blockIdx.x] = total;
        part[nblocks + blockIdx.x] = mm;
    }
}

// Exclusive prefix of the counts -> offsets; counts are reset to zero for the
// next call.  offsets[nbins] = number of particles.  Block 0 also writes
// stats[0] = largest (sub-)bin count and stats[1] = max |q| (from the
// particle-map partials); max |q| bounds the mesh charge of any point.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_apply(int nbins_, int nblocks, int* __restrict__ count,
                                                              const int* __restrict__ part,
                                                              int* __restrict__ offsets, int nqblocks,
                                                              const double* __restrict__ qpart,
                                                              double* __restrict__ stats)
{
    __shared__ int scratch[17];
    __shared__ int sbase;
    __shared__ double smax[2][SCAN_THREADS / 64];
    if (blockIdx.x == 0) {
        int mc = 0;
        double mq = 0.0;
        for (int j = threadIdx.x; j < nblocks; j += SCAN_THREADS) mc = max(mc, part[nblocks + j]);
        for (int j = threadIdx.x; j < nqblocks; j += SCAN_THREADS) mq = fmax(mq, qpart[3 * j + 2]);
        double mcd = (double)mc;
        for (int d = 32; d > 0; d >>= 1) {
            mcd = fmax(mcd, __shfl_down(mcd, d, 64));
            mq = fmax(mq, __shfl_down(mq, d, 64));
        }
        if ((threadIdx.x & 63) == 0) {
            smax[0][threadIdx.x >> 6] = mcd;
            smax[1][threadIdx.x >> 6] = mq;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double a = 0.0, b = 0.0;
            for (int w = 0; w < SCAN_THREADS / 64; ++w) {
                a = fmax(a, smax[0][w]);
                b = fmax(b, smax[1][w]);
            }
            stats[0] = a;
            stats[1] = b;
        }
    }
    // base of this chunk: sum of the chunks before it
    int pre = 0;
    for (int j = threadIdx.x; j < blockIdx.x; j += SCAN_THREADS) pre += part[j];
    int tot_pre;
    block_exclusive_scan(pre, scratch, &tot_pre);
    if (threadIdx.x == 0) sbase = tot_pre;
    __syncthreads();
    const int base = blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_ITEMS;
    int c[SCAN_ITEMS];
    int v = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        c[k] = (base + k < nbins_) ? count[base + k] : 0;
        v += c[k];
    }
    int total;
    int ex = block_exclusive_scan(v, scratch, &total) + sbase;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < nbins_) {
            offsets[base + k] = ex;
            count[base + k] = 0;
        }
        ex += c[k];
    }
    if (blockIdx.x == nblocks - 1 && threadIdx.x == 0) offsets[nbins_] = sbase + total;
}

template <typename TI, typename R>
__global__ __launch_bounds__(MAP_THREADS) void k_scatter(int n, const TI* __restrict__ pos,
                                                          const TI* __restrict__ q, MapGeo g,
                                                          const int* __restrict__ offsets,
                                                          const int* __restrict__ slot,
                                                          typename Rec<R>::T* __restrict__ rec,
                                                          int* __restrict__ perm)
{
    const int i = blockIdx.x * MAP_THREADS + threadIdx.x;
    if (i >= n) return;
    int s[3];
    double f[3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
        map_coord((double)pos[3 * (size_t)i + d], g.lo[d], g.h[d], g.K[d], g.shift, s[d], f[d]);
    int sl[3];
    const int dest = offsets[bin_of(g, s, sl) * NSUB + (i & (NSUB - 1))] + slot[i];
    typename Rec<R>::T r;
    r.x = (R)((double)sl[0] + f[0]);
    r.y = (R)((double)sl[1] + f[1]);
    r.z = (R)((double)sl[2] + f[2]);
    r.w = (R)q[i];
    rec[dest] = r;
    perm[dest] = i;
}

inline int grid_for(int64_t n, int threads) { return (int)((n + threads - 1) / threads); }

}  // namespace

hipError_t launch_map_count(pppm_plan_s* pl, int64_t n, const void* pos, const void* q)
{
    const int blocks = grid_for(n, MAP_THREADS);
    pl->qpart_blocks = blocks;
    if (blocks == 0) return hipGetLastError();
    if (pl->p.io_dtype == PPPM_F32)
        k_map_count<float><<<blocks, MAP_THREADS, 0, pl->stream>>>(
            (int)n, (const float*)pos, (const float*)q, pl->geo, pl->count, pl->slot, pl->qpart, pl->flags);
    else
        k_map_count<double><<<blocks, MAP_THREADS, 0, pl->stream>>>(
            (int)n, (const double*)pos, (const double*)q, pl->geo, pl->count, pl->slot, pl->qpart, pl->flags);
    return hipGetLastError();
}

hipError_t launch_scan(pppm_plan_s* pl)
{
    const int64_t nsub = pl->nbins * NSUB;
    const int nb = grid_for(nsub, SCAN_BLOCK);
    k_scan_reduce<<<nb, SCAN_THREADS, 0, pl->stream>>>((int)nsub, nb, pl->count, pl->scan_part);
    k_scan_apply<<<nb, SCAN_THREADS, 0, pl->stream>>>((int)nsub, nb, pl->count, pl->scan_part, pl->offsets,
                                                      (int)pl->qpart_blocks, pl->qpart, pl->eterms + 6);
    return hipGetLastError();
}

hipError_t launch_scatter(pppm_plan_s* pl, int64_t n, const void* pos, const void* q)
{
    const int blocks = grid_for(n, MAP_THREADS);
    if (blocks == 0) return hipGetLastError();
    const bool f32io = pl->p.io_dtype == PPPM_F32;
    if (pl->mixed) {
        auto* rec = (float4*)pl->records;
        if (f32io)
            k_scatter<float, float><<<blocks, MAP_THREADS, 0, pl->stream>>>(
                (int)n, (const float*)pos, (const float*)q, pl->geo, pl->offsets, pl->slot, rec, pl->perm);
        else
            k_scatter<double, float><<<blocks, MAP_THREADS, 0, pl->stream>>>(
                (int)n, (const double*)pos, (const double*)q, pl->geo, pl->offsets, pl->slot, rec, pl->perm);
    } else {
        auto* rec = (double4*)pl->records;
        if (f32io)
            k_scatter<float, double><<<blocks, MAP_THREADS, 0, pl->stream>>>(
                (int)n, (const float*)pos, (const float*)q, pl->geo, pl->offsets, pl->slot, rec, pl->perm);
        else
            k_scatter<double, double><<<blocks, MAP_THREADS, 0, pl->stream>>>(
                (int)n, (const double*)pos, (const double*)q, pl->geo, pl->offsets, pl->slot, rec, pl->perm);
    }
    return hipGetLastError();
}

}  // namespace pppm
