// Tile geometry shared by the binning, spread and gather kernels.
//
// The mesh is cut into tiles of B_x x B_y x B_z points; a charge belongs to
// the tile holding its stencil start and, within it, to one of 8 halo
// classes (bit d: the stencil reaches past the tile's upper face along d).
// The bins of a tile are laid out in the Gray-code class order
// 0, 1, 3, 2, 6, 7, 5, 4, which makes the classes a neighbouring tile needs
// from each lower neighbour (all classes containing the direction) fall into
// at most two contiguous ranges: a tile reads its own range plus at most 9
// halo ranges.
#pragma once

#include "device_common.h"

namespace pppm {

// bin position of each class within its tile
__host__ __device__ constexpr int class_pos(int c)
{
    return c == 0 ? 0 : c == 1 ? 1 : c == 2 ? 3 : c == 3 ? 2 : c == 4 ? 7 : c == 5 ? 6 : c == 6 ? 4 : 5;
}

// Runs a tile reads: direction mask (bit d: take the lower neighbour along d;
// 0 = the tile itself) and the bin-position range [first, last).
constexpr int NRUNS = 10;
__host__ __device__ constexpr int run_dir(int r)
{
    return r == 0 ? 0 : r <= 2 ? 1 : r == 3 ? 2 : r == 4 ? 4 : r <= 6 ? 3 : r == 7 ? 5 : r == 8 ? 6 : 7;
}
__host__ __device__ constexpr int run_first(int r)
{
    return r == 0 ? 0 : r == 1 ? 1 : r == 2 ? 5 : r == 3 ? 2 : r == 4 ? 4 : r == 5 ? 2 : r == 6 ? 5 : r == 7 ? 5 : r == 8 ? 4 : 5;
}
__host__ __device__ constexpr int run_last(int r)
{
    return r == 0 ? 8 : r == 1 ? 3 : r == 2 ? 7 : r == 3 ? 6 : r == 4 ? 8 : r == 5 ? 3 : r == 6 ? 6 : r == 7 ? 7 : r == 8 ? 6 : 6;
}

__device__ __forceinline__ void tile_coords(const MapGeo& g, int tile, int (&t)[3])
{
    t[0] = tile % g.ntile[0];
    t[1] = (tile / g.ntile[0]) % g.ntile[1];
    t[2] = tile / (g.ntile[0] * g.ntile[1]);
}

__device__ __forceinline__ int tile_extent(const MapGeo& g, int d, int t) { return min(g.B[d], g.K[d] - t * g.B[d]); }

// Run table of one tile in LDS (NRUNS + 1 entries; pre[NRUNS] = total).
struct RunTable {
    int start[NRUNS];
    int pre[NRUNS + 1];
    int shift[NRUNS];  // per axis, 8 bits each (biased by 128): tile coordinate of the record's tile origin
    int ext[NRUNS];    // per axis, 8 bits each: extent of the record's tile
};

// Built by the first wavefront; the caller synchronises before use.
__device__ __forceinline__ void build_run_table(const MapGeo& g, const int (&t)[3], const int* __restrict__ offsets,
                                                RunTable& rt)
{
    if (threadIdx.x >= 64) return;
    const int r = threadIdx.x;
    int cnt = 0, start = 0, shift = 0, ext = 0;
    if (r < NRUNS) {
        const int dir = run_dir(r);
        bool active = true;
        int tn[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const bool pull = (dir >> d) & 1;
            active &= !pull || g.ntile[d] >= 2;
            tn[d] = pull ? (t[d] == 0 ? g.ntile[d] - 1 : t[d] - 1) : t[d];
            const int e = tile_extent(g, d, tn[d]);
            ext |= e << (8 * d);
            shift |= ((pull ? -e : 0) + 128) << (8 * d);
        }
        if (active) {
            const int nb = (tn[2] * g.ntile[1] + tn[1]) * g.ntile[0] + tn[0];
            start = offsets[(nb * NCLASS + run_first(r)) * g.bin_stride];
            cnt = offsets[(nb * NCLASS + run_last(r)) * g.bin_stride] - start;
        }
    }
    const int inc = wave_inclusive_scan(cnt);
    if (r < NRUNS) {
        rt.start[r] = start;
        rt.pre[r] = inc - cnt;
        rt.shift[r] = shift;
        rt.ext[r] = ext;
    }
    if (r == NRUNS - 1) rt.pre[NRUNS] = inc;
}

__device__ __forceinline__ int find_run(const RunTable& rt, int v)
{
    int r = 0;
#pragma unroll
    for (int k = 1; k < NRUNS; ++k) r += (rt.pre[k] <= v) ? 1 : 0;
    return r;
}

// Decode one axis of a record: t = stencil start within its tile + fraction.
// The particle map stores t below s + 1, so the integer part is the start it
// chose; the clamp to the tile is a guard.
template <typename R>
__device__ __forceinline__ void decode_local(R t, int ext, int& s, R& f)
{
    int si = (int)t;
    si = si < 0 ? 0 : (si > ext - 1 ? ext - 1 : si);
    s = si;
    f = t - R(si);
}

}  // namespace pppm
