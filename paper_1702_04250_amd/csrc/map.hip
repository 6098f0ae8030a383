// Particle map (the per-atom part of the mapping functions, paper Section
// 3.1): wrap each charge into the box, find its stencil start and fraction,
// and counting-sort the charges by the mesh sub-brick that holds their
// stencil start.  Three passes: count (with per-sub-brick rank), scan,
// scatter into binned order.
#include "device_common.h"

namespace pppm {

namespace {

template <typename TI>
__global__ __launch_bounds__(MAP_THREADS) void k_map_count(int n, const TI* __restrict__ pos,
                                                            const TI* __restrict__ q, MapGeo g,
                                                            int* __restrict__ count,
                                                            int* __restrict__ slot,
                                                            double* __restrict__ qpart,
                                                            int* __restrict__ flags)
{
    __shared__ double red[2][MAP_THREADS / 64];
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
        const int id = ((s[2] / SB) * g.nsb[1] + s[1] / SB) * g.nsb[0] + s[0] / SB;
        slot[i] = atomicAdd(&count[id], 1);
    }
    // charge sums for the self and background energy terms
    double a = qi, b = qi * qi;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        a += __shfl_down(a, d, 64);
        b += __shfl_down(b, d, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wid] = a;
        red[1][wid] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0;
        for (int w = 0; w < MAP_THREADS / 64; ++w) {
            sa += red[0][w];
            sb += red[1][w];
        }
        qpart[2 * blockIdx.x] = sa;
        qpart[2 * blockIdx.x + 1] = sb;
    }
}

// Sum of each SCAN_BLOCK-long chunk of the sub-brick counts.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(int nsub, const int* __restrict__ count,
                                                               int* __restrict__ part)
{
    __shared__ int scratch[17];
    const int base = blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_ITEMS;
    int v = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k)
        if (base + k < nsub) v += count[base + k];
    int total;
    block_exclusive_scan(v, scratch, &total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// Exclusive prefix of the counts -> offsets; counts are reset to zero for the
// next call.  offsets[nsub] = number of particles.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_apply(int nsub, int nblocks, int* __restrict__ count,
                                                              const int* __restrict__ part,
                                                              int* __restrict__ offsets)
{
    __shared__ int scratch[17];
    __shared__ int sbase;
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
        c[k] = (base + k < nsub) ? count[base + k] : 0;
        v += c[k];
    }
    int total;
    int ex = block_exclusive_scan(v, scratch, &total) + sbase;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < nsub) {
            offsets[base + k] = ex;
            count[base + k] = 0;
        }
        ex += c[k];
    }
    if (blockIdx.x == nblocks - 1 && threadIdx.x == 0) offsets[nsub] = sbase + total;
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
    const int id = ((s[2] / SB) * g.nsb[1] + s[1] / SB) * g.nsb[0] + s[0] / SB;
    const int dest = offsets[id] + slot[i];
    typename Rec<R>::T r;
    r.x = (R)((double)(s[0] % SB) + f[0]);
    r.y = (R)((double)(s[1] % SB) + f[1]);
    r.z = (R)((double)(s[2] % SB) + f[2]);
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
    const int nb = grid_for(pl->nsub, SCAN_BLOCK);
    k_scan_reduce<<<nb, SCAN_THREADS, 0, pl->stream>>>((int)pl->nsub, pl->count, pl->scan_part);
    k_scan_apply<<<nb, SCAN_THREADS, 0, pl->stream>>>((int)pl->nsub, nb, pl->count, pl->scan_part, pl->offsets);
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
