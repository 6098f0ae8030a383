// Particle map (the per-atom part of the mapping functions, paper Section
// 3.1): wrap each charge into the box, find its stencil start and fraction,
// and counting-sort the charges by (tile, halo class) bin.  Passes: count
// (with a rank per charge), scan, scatter into binned order.
//
// Two forms of the count.  Histogram form (bins fit in LDS): block b bins a
// chunk of consecutive charges in an LDS histogram, ranking each charge with
// an LDS atomic; a column pass turns the per-block counts into per-block
// offsets within each bin.  Device-scope atomics are avoided: on a chip whose
// XCDs have separate L2 caches they are resolved past the L2 and throttle a
// counting pass over half a million charges.  Atomic form (otherwise): one
// device-scope atomic per charge on one of NSUB sub-bins of its bin.
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

// Block-wide sums of q and q^2 and max |q| into qpart[3 * blockIdx.x ..].
template <int THREADS>
__device__ __forceinline__ void charge_sums(double a, double b, double c, double* __restrict__ qpart)
{
    __shared__ double red[3][THREADS / 64];
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
        for (int w = 0; w < THREADS / 64; ++w) {
            sa += red[0][w];
            sb += red[1][w];
            sc = fmax(sc, red[2][w]);
        }
        qpart[3 * blockIdx.x] = sa;
        qpart[3 * blockIdx.x + 1] = sb;
        qpart[3 * blockIdx.x + 2] = sc;
    }
}

template <typename TI>
__global__ __launch_bounds__(MAP_THREADS) void k_map_count(int n, const TI* __restrict__ pos,
                                                            const TI* __restrict__ q, MapGeo g,
                                                            int* __restrict__ count,
                                                            int* __restrict__ slot,
                                                            double* __restrict__ qpart,
                                                            int* __restrict__ flags)
{
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
    charge_sums<MAP_THREADS>(qi, qi * qi, fabs(qi), qpart);
}

// Histogram count: block b maps charges [b * chunk, (b + 1) * chunk) and
// counts them per bin in LDS; slot[i] = rank of charge i among the block's
// charges of its bin; hist[b][bin] = the block's count.
template <typename TI>
__global__ __launch_bounds__(HIST_THREADS) void k_hist_count(int n, int chunk, int nbins, const TI* __restrict__ pos,
                                                              const TI* __restrict__ q, MapGeo g,
                                                              int* __restrict__ slot, int* __restrict__ hist,
                                                              double* __restrict__ qpart, int* __restrict__ flags)
{
    extern __shared__ int lhist[];
    for (int b = threadIdx.x; b < nbins; b += HIST_THREADS) lhist[b] = 0;
    __syncthreads();
    const int i0 = blockIdx.x * chunk;
    const int i1 = min(n, i0 + chunk);
    double a = 0.0, b2 = 0.0, c = 0.0;
    // up to four charges per thread per pass, their loads issued together
    constexpr int U = 4;
    for (int ib = i0 + threadIdx.x; ib < i1; ib += U * HIST_THREADS) {
        TI x[U][3], qq[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = ib + u * HIST_THREADS;
            if (i < i1) {
#pragma unroll
                for (int d = 0; d < 3; ++d) x[u][d] = pos[3 * (size_t)i + d];
                qq[u] = q[i];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = ib + u * HIST_THREADS;
            if (i >= i1) break;
            int s[3];
            double f[3];
            bool ok = true;
#pragma unroll
            for (int d = 0; d < 3; ++d) ok &= map_coord((double)x[u][d], g.lo[d], g.h[d], g.K[d], g.shift, s[d], f[d]);
            const double qi = (double)qq[u];
            if (!isfinite(qi)) ok = false;
            if (!ok && g.check_finite) atomicOr(flags, 1);
            int sl[3];
            slot[i] = atomicAdd(&lhist[bin_of(g, s, sl)], 1);
            a += qi;
            b2 += qi * qi;
            c = fmax(c, fabs(qi));
        }
    }
    charge_sums<HIST_THREADS>(a, b2, c, qpart);  // synchronises the block
    int* __restrict__ row = hist + (size_t)blockIdx.x * nbins;
    for (int b = threadIdx.x; b < nbins; b += HIST_THREADS) row[b] = lhist[b];
}

// Column pass.  A workgroup takes PREFIX_BINS bins and splits the histogram
// blocks into PREFIX_SEGS segments: thread (bin, segment) holds its
// segment's counts in registers, the segment sums are combined through LDS,
// and the counts become their exclusive prefix over blocks (the block's
// offset within the bin); the bin total goes to count[bin].  512 threads in
// 16 segments of at most 16 blocks: the pass is latency bound, and shorter
// per-thread chains in wider workgroups finish sooner (particle map of
// 524,288 charges on 4,096 bins: 28.7 us against 29.7 us with 256 threads
// in 8 segments; 30.5 us with 512 threads in 32 segments, 30.6 us with 256
// in 16).
constexpr int PREFIX_THREADS = 512;
constexpr int PREFIX_SEGS = 16;
constexpr int PREFIX_BINS = PREFIX_THREADS / PREFIX_SEGS;
constexpr int PREFIX_SEG_MAX = HIST_MAX_BLOCKS / PREFIX_SEGS;

__global__ __launch_bounds__(PREFIX_THREADS) void k_hist_prefix(int nbins, int nblocks, int* __restrict__ hist,
                                                                 int* __restrict__ count)
{
    __shared__ int segsum[PREFIX_SEGS][PREFIX_BINS];
    const int lb = threadIdx.x % PREFIX_BINS, seg = threadIdx.x / PREFIX_BINS;
    const int b = blockIdx.x * PREFIX_BINS + lb;
    const int seglen = (nblocks + PREFIX_SEGS - 1) / PREFIX_SEGS;
    const int k0 = seg * seglen, k1 = min(nblocks, k0 + seglen);
    int v[PREFIX_SEG_MAX];
    int sum = 0;
#pragma unroll
    for (int u = 0; u < PREFIX_SEG_MAX; ++u) {
        v[u] = (b < nbins && k0 + u < k1) ? hist[(size_t)(k0 + u) * nbins + b] : 0;
        sum += v[u];
    }
    segsum[seg][lb] = sum;
    __syncthreads();
    int run = 0, bin_total = 0;
#pragma unroll
    for (int s2 = 0; s2 < PREFIX_SEGS; ++s2) {
        const int x = segsum[s2][lb];
        run += (s2 < seg) ? x : 0;
        bin_total += x;
    }
    if (b < nbins) {
#pragma unroll
        for (int u = 0; u < PREFIX_SEG_MAX; ++u)
            if (k0 + u < k1) {
                hist[(size_t)(k0 + u) * nbins + b] = run;
                run += v[u];
            }
        if (seg == 0) count[b] = bin_total;
    }
}

// Single-workgroup exclusive scan of the bin totals (nbins <= HIST_MAX_BINS)
// into offsets[0 .. nbins]; zeroes count again; stats[0] = largest bin,
// stats[1] = max |q| and stats[2] = sum q^2 from the count pass's partials.
constexpr int SSCAN_THREADS = 1024;
constexpr int SSCAN_PER = HIST_MAX_BINS / SSCAN_THREADS;

__global__ __launch_bounds__(SSCAN_THREADS) void k_scan_single(int nbins, int* __restrict__ count,
                                                                int* __restrict__ offsets, int nqblocks,
                                                                const double* __restrict__ qpart,
                                                                double* __restrict__ stats)
{
    __shared__ int scratch[17];
    __shared__ double smax[3][SSCAN_THREADS / 64];
    const int per = (nbins + SSCAN_THREADS - 1) / SSCAN_THREADS;  // <= SSCAN_PER
    const int j0 = threadIdx.x * per;
    int c[SSCAN_PER];
    int sum = 0, mc = 0;
#pragma unroll
    for (int u = 0; u < SSCAN_PER; ++u) {
        c[u] = (u < per && j0 + u < nbins) ? count[j0 + u] : 0;
        sum += c[u];
        mc = max(mc, c[u]);
    }
    int total;
    int ex = block_exclusive_scan(sum, scratch, &total);
#pragma unroll
    for (int u = 0; u < SSCAN_PER; ++u)
        if (u < per && j0 + u < nbins) {
            offsets[j0 + u] = ex;
            ex += c[u];
            count[j0 + u] = 0;
        }
    double mq = 0.0, sq = 0.0;
    for (int j = threadIdx.x; j < nqblocks; j += SSCAN_THREADS) {
        mq = fmax(mq, qpart[3 * j + 2]);
        sq += qpart[3 * j + 1];
    }
    double mcd = (double)mc;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        mcd = fmax(mcd, __shfl_down(mcd, d, 64));
        mq = fmax(mq, __shfl_down(mq, d, 64));
        sq += __shfl_down(sq, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        smax[0][threadIdx.x >> 6] = mcd;
        smax[1][threadIdx.x >> 6] = mq;
        smax[2][threadIdx.x >> 6] = sq;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0.0, y = 0.0, z = 0.0;
        for (int w = 0; w < SSCAN_THREADS / 64; ++w) {
            x = fmax(x, smax[0][w]);
            y = fmax(y, smax[1][w]);
            z += smax[2][w];
        }
        stats[0] = x;
        stats[1] = y;
        stats[2] = z;
        offsets[nbins] = total;
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
// stats[0] = largest (sub-)bin count, stats[1] = max |q| and stats[2] =
// sum q^2 (from the
// particle-map partials); max |q| bounds the mesh charge of any point.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_apply(int nbins_, int nblocks, int* __restrict__ count,
                                                              const int* __restrict__ part,
                                                              int* __restrict__ offsets, int nqblocks,
                                                              const double* __restrict__ qpart,
                                                              double* __restrict__ stats)
{
    __shared__ int scratch[17];
    __shared__ int sbase;
    __shared__ double smax[3][SCAN_THREADS / 64];
    if (blockIdx.x == 0) {
        int mc = 0;
        double mq = 0.0, sq = 0.0;
        for (int j = threadIdx.x; j < nblocks; j += SCAN_THREADS) mc = max(mc, part[nblocks + j]);
        for (int j = threadIdx.x; j < nqblocks; j += SCAN_THREADS) {
            mq = fmax(mq, qpart[3 * j + 2]);
            sq += qpart[3 * j + 1];
        }
        double mcd = (double)mc;
        for (int d = 32; d > 0; d >>= 1) {
            mcd = fmax(mcd, __shfl_down(mcd, d, 64));
            mq = fmax(mq, __shfl_down(mq, d, 64));
            sq += __shfl_down(sq, d, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            smax[0][threadIdx.x >> 6] = mcd;
            smax[1][threadIdx.x >> 6] = mq;
            smax[2][threadIdx.x >> 6] = sq;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double a = 0.0, b = 0.0, c = 0.0;
            for (int w = 0; w < SCAN_THREADS / 64; ++w) {
                a = fmax(a, smax[0][w]);
                b = fmax(b, smax[1][w]);
                c += smax[2][w];
            }
            stats[0] = a;
            stats[1] = b;
            stats[2] = c;
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

// A record coordinate t = s + f stored in R: when f is within half an R step
// of 1, t rounds up to s + 1, and the kernels would decode the next point as
// the stencil start.  The order-2 ad derivative weights jump there, so the
// value is kept one step below s + 1 instead (f changes by at most one step
// of t), and every kernel decodes the start the map chose.
__device__ __forceinline__ float below_next(float t, int s)
{
    const float lim = (float)(s + 1);
    return t < lim ? t : __int_as_float(__float_as_int(lim) - 1);
}
__device__ __forceinline__ double below_next(double t, int s)
{
    const double lim = (double)(s + 1);
    return t < lim ? t : __longlong_as_double(__double_as_longlong(lim) - 1);
}

// Scatter into binned order.  Histogram form (hist != nullptr): destination
// = bin offset + the block's offset within the bin + rank; atomic form:
// sub-bin offset + rank.
// The binned record of charge i, written at dest_of(bin): stencil start
// within the tile plus fraction per axis, and the charge.
template <typename TI, typename R, typename Dest>
__device__ __forceinline__ void scatter_charge(int i, const TI* __restrict__ pos, const TI* __restrict__ q,
                                               const MapGeo& g, Dest dest_of, typename Rec<R>::T* __restrict__ rec,
                                               int* __restrict__ perm)
{
    int s[3];
    double f[3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
        map_coord((double)pos[3 * (size_t)i + d], g.lo[d], g.h[d], g.K[d], g.shift, s[d], f[d]);
    int sl[3];
    const int bin = bin_of(g, s, sl);
    const int dest = dest_of(bin);
    if (g.wtab) {
        // tabulated weights: the nearest table node is chosen here, in FP64
        // (the record keeps the node's fraction, from which the kernels
        // recover the same entry in either precision)
#pragma unroll
        for (int d = 0; d < 3; ++d) f[d] = floor(f[d] * (double)g.wtab_n + 0.5) / (double)g.wtab_n;
    }
    typename Rec<R>::T r;
    r.x = below_next((R)((double)sl[0] + f[0]), sl[0]);
    r.y = below_next((R)((double)sl[1] + f[1]), sl[1]);
    r.z = below_next((R)((double)sl[2] + f[2]), sl[2]);
    r.w = (R)q[i];
    rec[dest] = r;
    perm[dest] = i;
}

template <typename TI, typename R>
__global__ __launch_bounds__(MAP_THREADS) void k_scatter(int n, const TI* __restrict__ pos,
                                                          const TI* __restrict__ q, MapGeo g,
                                                          const int* __restrict__ offsets,
                                                          const int* __restrict__ slot,
                                                          const int* __restrict__ hist, int chunk, int nbins,
                                                          typename Rec<R>::T* __restrict__ rec,
                                                          int* __restrict__ perm)
{
    // the blocks that read one histogram row (HIST_CHUNK charges) run on one
    // XCD, so that row is fetched into one L2 only
    const int i = xcd_remap<HIST_CHUNK / MAP_THREADS>(blockIdx.x, gridDim.x) * MAP_THREADS + threadIdx.x;
    if (i >= n) return;
    scatter_charge<TI, R>(
        i, pos, q, g,
        [&](int bin) {
            return hist ? offsets[bin] + hist[(size_t)(i / chunk) * nbins + bin] + slot[i]
                        : offsets[bin * NSUB + (i & (NSUB - 1))] + slot[i];
        },
        rec, perm);
}

// Histogram form with at most FUSED_SCAN_MAX_BINS bins: one block per
// histogram chunk scans the bin totals itself (a few KiB, read from L2)
// into LDS and scatters its chunk with them; block 0 also publishes
// offsets[0 .. nbins] and the statistics, as the single-block scan would.
// This saves that kernel's launch.  Consecutive chunks write adjacent
// records of every bin, so each XCD takes one contiguous run of chunks:
// a record line is then filled within one L2 instead of being written back
// in parts from several.
constexpr int FUSED_SCAN_MAX_BINS = 8192;

template <typename TI, typename R>
__global__ __launch_bounds__(HIST_THREADS) void k_scatter_scan(int n, int chunk, int nbins, const TI* __restrict__ pos,
                                                                const TI* __restrict__ q, MapGeo g,
                                                                const int* __restrict__ count,
                                                                int* __restrict__ offsets,
                                                                const int* __restrict__ slot,
                                                                const int* __restrict__ hist, int nqblocks,
                                                                const double* __restrict__ qpart,
                                                                double* __restrict__ stats,
                                                                typename Rec<R>::T* __restrict__ rec,
                                                                int* __restrict__ perm)
{
    extern __shared__ int loff[];  // [nbins] exclusive prefix of the bin totals
    __shared__ int scratch[17];
    __shared__ double smax[3][HIST_THREADS / 64];
    constexpr int PER = FUSED_SCAN_MAX_BINS / HIST_THREADS;
    const int per = (nbins + HIST_THREADS - 1) / HIST_THREADS;  // <= PER
    const int j0 = threadIdx.x * per;
    int c[PER];
    int sum = 0, mc = 0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        c[u] = (u < per && j0 + u < nbins) ? count[j0 + u] : 0;
        sum += c[u];
        mc = max(mc, c[u]);
    }
    int total;
    int ex = block_exclusive_scan(sum, scratch, &total);
    const bool pub = blockIdx.x == 0;
#pragma unroll
    for (int u = 0; u < PER; ++u)
        if (u < per && j0 + u < nbins) {
            loff[j0 + u] = ex;
            if (pub) offsets[j0 + u] = ex;
            ex += c[u];
        }
    if (pub) {
        // largest bin and largest |q| (from the count pass's partials)
        double mq = 0.0, sq = 0.0;
        for (int j = threadIdx.x; j < nqblocks; j += HIST_THREADS) {
            mq = fmax(mq, qpart[3 * j + 2]);
            sq += qpart[3 * j + 1];
        }
        double mcd = (double)mc;
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) {
            mcd = fmax(mcd, __shfl_down(mcd, d, 64));
            mq = fmax(mq, __shfl_down(mq, d, 64));
            sq += __shfl_down(sq, d, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            smax[0][threadIdx.x >> 6] = mcd;
            smax[1][threadIdx.x >> 6] = mq;
            smax[2][threadIdx.x >> 6] = sq;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double x = 0.0, y = 0.0, z = 0.0;
            for (int w = 0; w < HIST_THREADS / 64; ++w) {
                x = fmax(x, smax[0][w]);
                y = fmax(y, smax[1][w]);
                z += smax[2][w];
            }
            stats[0] = x;
            stats[1] = y;
            stats[2] = z;
            offsets[nbins] = total;
        }
    }
    __syncthreads();
    const int cb = xcd_contiguous(blockIdx.x, gridDim.x);
    const int i0 = cb * chunk, i1 = min(n, i0 + chunk);
    const int* __restrict__ row = hist + (size_t)cb * nbins;
    for (int i = i0 + (int)threadIdx.x; i < i1; i += HIST_THREADS)
        scatter_charge<TI, R>(
            i, pos, q, g, [&](int bin) { return loff[bin] + row[bin] + slot[i]; }, rec, perm);
}

inline int grid_for(int64_t n, int threads) { return (int)((n + threads - 1) / threads); }

}  // namespace

hipError_t launch_map_count(pppm_plan_s* pl, int64_t n, const void* pos, const void* q)
{
    if (pl->geo.bin_stride == 1) {
        // histogram form: about HIST_CHUNK charges per block
        const int nbins = (int)pl->nbins;
        int nb = (int)((n + HIST_CHUNK - 1) / HIST_CHUNK);
        nb = nb < 1 ? 1 : (nb > HIST_MAX_BLOCKS ? HIST_MAX_BLOCKS : nb);
        const int chunk = (int)((n + nb - 1) / nb);
        pl->hist_blocks = nb;
        pl->hist_chunk = chunk > 0 ? chunk : 1;
        pl->qpart_blocks = nb;
        const size_t lds = (size_t)nbins * sizeof(int);
        if (pl->p.io_dtype == PPPM_F32)
            k_hist_count<float><<<nb, HIST_THREADS, lds, pl->stream>>>(
                (int)n, pl->hist_chunk, nbins, (const float*)pos, (const float*)q, pl->geo, pl->slot, pl->hist,
                pl->qpart, pl->flags);
        else
            k_hist_count<double><<<nb, HIST_THREADS, lds, pl->stream>>>(
                (int)n, pl->hist_chunk, nbins, (const double*)pos, (const double*)q, pl->geo, pl->slot, pl->hist,
                pl->qpart, pl->flags);
        k_hist_prefix<<<grid_for(nbins, PREFIX_BINS), PREFIX_THREADS, 0, pl->stream>>>(nbins, nb, pl->hist,
                                                                                          pl->count);
        if (nbins > FUSED_SCAN_MAX_BINS)  // else the scatter scans (k_scatter_scan)
            k_scan_single<<<1, SSCAN_THREADS, 0, pl->stream>>>(nbins, pl->count, pl->offsets, nb, pl->qpart,
                                                               pl->eterms + 6);
        return hipGetLastError();
    }
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
    if (pl->geo.bin_stride == 1) return hipGetLastError();  // scanned by the histogram count
    const int64_t nsub = pl->nbins * pl->geo.bin_stride;
    const int nb = grid_for(nsub, SCAN_BLOCK);
    k_scan_reduce<<<nb, SCAN_THREADS, 0, pl->stream>>>((int)nsub, nb, pl->count, pl->scan_part);
    k_scan_apply<<<nb, SCAN_THREADS, 0, pl->stream>>>((int)nsub, nb, pl->count, pl->scan_part, pl->offsets,
                                                      (int)pl->qpart_blocks, pl->qpart, pl->eterms + 6);
    return hipGetLastError();
}

template <typename TI, typename R>
void launch_scatter_scan(pppm_plan_s* pl, int64_t n, const void* pos, const void* q)
{
    const int nbins = (int)pl->nbins;
    k_scatter_scan<TI, R><<<pl->hist_blocks, HIST_THREADS, (size_t)nbins * sizeof(int), pl->stream>>>(
        (int)n, pl->hist_chunk, nbins, (const TI*)pos, (const TI*)q, pl->geo, pl->count, pl->offsets, pl->slot,
        pl->hist, (int)pl->qpart_blocks, pl->qpart, pl->eterms + 6, (typename Rec<R>::T*)pl->records, pl->perm);
}

hipError_t launch_scatter(pppm_plan_s* pl, int64_t n, const void* pos, const void* q)
{
    if (pl->geo.bin_stride == 1 && pl->nbins <= FUSED_SCAN_MAX_BINS) {
        // also publishes the offsets when n == 0 (one block at least)
        const bool f32io = pl->p.io_dtype == PPPM_F32;
        if (pl->mixed)
            f32io ? launch_scatter_scan<float, float>(pl, n, pos, q) : launch_scatter_scan<double, float>(pl, n, pos, q);
        else
            f32io ? launch_scatter_scan<float, double>(pl, n, pos, q)
                  : launch_scatter_scan<double, double>(pl, n, pos, q);
        return hipGetLastError();
    }
    const int blocks = grid_for(n, MAP_THREADS);
    if (blocks == 0) return hipGetLastError();
    const bool f32io = pl->p.io_dtype == PPPM_F32;
    const bool h = pl->geo.bin_stride == 1;
    const int* hist = h ? pl->hist : nullptr;
    const int chunk = h ? pl->hist_chunk : 1, nbins = (int)pl->nbins;
    if (pl->mixed) {
        auto* rec = (float4*)pl->records;
        if (f32io)
            k_scatter<float, float><<<blocks, MAP_THREADS, 0, pl->stream>>>(
                (int)n, (const float*)pos, (const float*)q, pl->geo, pl->offsets, pl->slot, hist, chunk, nbins, rec, pl->perm);
        else
            k_scatter<double, float><<<blocks, MAP_THREADS, 0, pl->stream>>>(
                (int)n, (const double*)pos, (const double*)q, pl->geo, pl->offsets, pl->slot, hist, chunk, nbins, rec, pl->perm);
    } else {
        auto* rec = (double4*)pl->records;
        if (f32io)
            k_scatter<float, double><<<blocks, MAP_THREADS, 0, pl->stream>>>(
                (int)n, (const float*)pos, (const float*)q, pl->geo, pl->offsets, pl->slot, hist, chunk, nbins, rec, pl->perm);
        else
            k_scatter<double, double><<<blocks, MAP_THREADS, 0, pl->stream>>>(
                (int)n, (const double*)pos, (const double*)q, pl->geo, pl->offsets, pl->slot, hist, chunk, nbins, rec, pl->perm);
    }
    return hipGetLastError();
}

}  // namespace pppm
