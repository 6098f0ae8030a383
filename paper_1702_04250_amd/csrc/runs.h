// Run tables: the list of sub-bricks (and their binned particle ranges) a
// workgroup tile reads, shared by the spread and gather kernels.
#pragma once

#include "device_common.h"

namespace pppm {

constexpr int MAXL = 24;  // sub-bricks one tile reads along one axis


// Sub-bricks along one axis whose stencil starts reach tile [T0, T0 + ext):
// starts in [T0 - (P - 1), T0 + ext - 1] modulo K.
__device__ inline int axis_subbricks(int T0, int ext, int K, int nsb, int halo, int* out)
{
    int cnt = 0;
    if (ext + halo >= K) {
        for (int i = 0; i < nsb && cnt < MAXL; ++i) out[cnt++] = i;
        return cnt;
    }
    int s = T0 - halo;
    if (s < 0) s += K;
    for (int c = 0; c < ext + halo; ++c) {
        const int sbi = s / SB;
        bool seen = false;
        for (int k = 0; k < cnt; ++k) seen |= (out[k] == sbi);
        if (!seen && cnt < MAXL) out[cnt++] = sbi;
        if (++s == K) s = 0;
    }
    return cnt;
}

// Build the run table (one run per sub-brick) in LDS and return the number
// of runs; prefix[r] is the exclusive prefix of the runs' particle counts and
// prefix[nruns] the total.
__device__ inline int build_runs(const TileGeo& tg, const int T0[3], const int ext[3], int halo,
                          const int* __restrict__ offsets, int* lists, int* cnts, int* run_start,
                          int* prefix, int* run_sb, int* scratch)
{
    if (threadIdx.x < 3) {
        const int d = threadIdx.x;
        cnts[d] = axis_subbricks(T0[d], ext[d], tg.K[d], tg.nsb[d], halo, lists + d * MAXL);
    }
    __syncthreads();
    const int nx = cnts[0], ny = cnts[1], nz = cnts[2];
    const int nruns = nx * ny * nz;
    if (nruns > MAX_RUNS) return -1;  // uniform over the workgroup; the host never launches this
    const int per = (nruns + blockDim.x - 1) / blockDim.x;
    const int r0 = threadIdx.x * per;
    int local = 0;
    for (int k = 0; k < per; ++k) {
        const int r = r0 + k;
        if (r < nruns) {
            const int ix = r % nx, iy = (r / nx) % ny, iz = r / (nx * ny);
            const int sx = lists[ix], sy = lists[MAXL + iy], sz = lists[2 * MAXL + iz];
            const int id = (sz * tg.nsb[1] + sy) * tg.nsb[0] + sx;
            const int st = offsets[id];
            const int c = offsets[id + 1] - st;
            run_start[r] = st;
            run_sb[r] = sx | (sy << 10) | (sz << 20);
            prefix[r] = c;  // count for now
            local += c;
        }
    }
    int total;
    int ex = block_exclusive_scan(local, scratch, &total);
    for (int k = 0; k < per; ++k) {
        const int r = r0 + k;
        if (r < nruns) {
            const int c = prefix[r];
            prefix[r] = ex;
            ex += c;
        }
    }
    if (threadIdx.x == 0) prefix[nruns] = total;
    __syncthreads();
    return nruns;
}

__device__ __forceinline__ int find_run(const int* prefix, int nruns, int v)
{
    // last r with prefix[r] <= v
    int lo = 0, hi = nruns;  // answer in [lo, hi)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= v) lo = mid; else hi = mid;
    }
    return lo;
}

}  // namespace pppm
