// fieldforce: the paper's Distribute-Force (Section 3.1), ik and ad modes,
// and the adjoint gather of the energy backward.
//
//   ik:      F_i = q_i sum_{P^3} wx wy wz (Ex, Ey, Ez)_m
//   ad:      F_i = -q_i (sum dwx wy wz phi / hx, sum wx dwy wz phi / hy,
//                        sum wx wy dwz phi / hz)
//   adjoint: dE/dr_i = q_i grad phi(r_i),
//            dE/dq_i = phi(r_i) - 2 C g q_i / sqrt(pi) - C pi Q / (V g^2),
//            both times dL/dE.
//
// GPU design: one workgroup per mesh tile.  The tile plus its P - 1 upper
// halo points of every field mesh is staged in LDS with coalesced loads,
// then each thread takes one binned charge of the tile's own sub-bricks,
// evaluates its stencil coefficients in registers and sums the P^3 staged
// values: rows along x first (unit stride, the paper's inner loop), then
// rows into planes, planes into the result (the "split atom" idea of the ad
// kernel: the per-atom epilogue is a few register operations).  Results are
// written straight to the caller's particle order through the permutation.
#include "tiles.h"

namespace pppm {

namespace {

struct GatherArgs {
    MapGeo g;
    const int* offsets;
    const void* rec;
    const int* perm;
    const void* field;   // ncomp meshes of type R, each ncell long
    long long ncell;
    int pitch_x;         // LDS row pitch
    int rows_y;          // LDS rows per plane
    double inv_h[3];
    void* out0;          // forces (ik/ad) or grad_pos (adjoint); N x 3
    void* out1;          // grad_q (adjoint); N
    const double* grad_energy;
    const double* eterms;
    double self_coef;    // 2 C g / sqrt(pi)
    double bg_coef;      // C pi / (V g^2)
    int vec_stage;       // tile origins and K_x allow 16-byte staging loads
    int sort_off;        // byte offset of the lane-assignment buffers in LDS
    const double* sfc;   // ad self-force coefficients of the stencil fraction's sines, or null
};

// sin(2 pi x) for x in [0, 2].  FP32: the hardware sine, whose argument is
// in turns (v_sin_f32); the ad self-force term it serves is a small
// correction, and on lone charges (whose force is all self-force) the
// corrections it gives match the FP64 ones to about 2e-6.  FP64: sinpi.
__device__ __forceinline__ float sin_turns(float x) { return __builtin_amdgcn_sinf(x); }
__device__ __forceinline__ double sin_turns(double x) { return sinpi(2.0 * x); }

// A value that is the same in every lane, moved to a scalar register.
__device__ __forceinline__ float uniform(float x)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ double uniform(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL)), hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <typename R> struct Vec16;
template <> struct Vec16<float> { using T = float4; };
template <> struct Vec16<double> { using T = double2; };

// Largest workgroup of a gather: 1024 threads for the mixed ik gather (its
// three staged meshes leave one workgroup per CU, so a wider one keeps more
// wavefronts in flight), 512 otherwise.  The plan's limits follow these.
__host__ __device__ constexpr int gather_threads_max(int mode, int real_bytes)
{
    return (mode == GATHER_IK && real_bytes == 4) ? 1024 : 512;
}

template <int P, int MODE, typename R, typename TO, bool TAB>
__global__ __launch_bounds__(gather_threads_max(MODE, sizeof(R))) void k_gather(GatherArgs a)
{
    constexpr int NC = (MODE == GATHER_IK) ? 3 : 1;
    constexpr bool DERIV = (MODE != GATHER_IK);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const MapGeo& g = a.g;

    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    int t[3];
    tile_coords(g, tile, t);
    const int T0[3] = {t[0] * g.B[0], t[1] * g.B[1], t[2] * g.B[2]};
    const int ext[3] = {tile_extent(g, 0, t[0]), tile_extent(g, 1, t[1]), tile_extent(g, 2, t[2])};
    const int first = a.offsets[tile * NCLASS * g.bin_stride], last = a.offsets[(tile + 1) * NCLASS * g.bin_stride];

    R* fld = (R*)smem_raw;
    const int plane = a.pitch_x * a.rows_y;
    const int nsl = plane * (g.B[2] + P - 1);  // one staged mesh
    const R* __restrict__ fg = (const R*)a.field;

    // The thread's first charge (record and caller index) is loaded before
    // the field is staged.
    using RT = typename Rec<R>::T;
    const RT* __restrict__ rec = (const RT*)a.rec;
    RT pr{};
    int pm = 0;
    if (first + (int)threadIdx.x < last) {
        pr = rec[first + threadIdx.x];
        if (sizeof(R) == 4) pm = a.perm[first + threadIdx.x];
    }

    // stage tile + upper halo of every field mesh (periodic wrap)
    if (a.vec_stage) {
        // 16-byte loads: rows start at multiples of 4 points and K_x % 4 == 0,
        // so a 4-point chunk never straddles the periodic wrap
        constexpr int VW = 16 / (int)sizeof(R);  // points per 16-byte chunk
        using V = typename Vec16<R>::T;
        const int sx = ext[0] + P - 1, sy = ext[1] + P - 1, sz = ext[2] + P - 1;
        const int nch = (sx + VW - 1) / VW;  // chunks per row
        const int n = nch * sy * sz;
        // all of a thread's chunks in flight before the first LDS store (one
        // round trip for the 1-mesh forms at P <= 7 and 512 threads)
        constexpr int U = NC == 1 ? 8 : 3;
        for (int i0 = 0; i0 < n; i0 += U * blockDim.x) {
            V v[U][NC];
            int li[U], nv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * blockDim.x + threadIdx.x;
                li[u] = -1;
                nv[u] = 0;
                if (i < n) {
                    const int cx = i % nch, ly = (i / nch) % sy, lz = i / (nch * sy);
                    const int lx = cx * VW;
                    int gx = T0[0] + lx, gy = T0[1] + ly, gz = T0[2] + lz;
                    if (gx >= g.K[0]) gx -= g.K[0];
                    if (gy >= g.K[1]) gy -= g.K[1];
                    if (gz >= g.K[2]) gz -= g.K[2];
                    const size_t gi = ((size_t)gz * g.K[1] + gy) * g.K[0] + gx;
                    li[u] = lz * plane + ly * a.pitch_x + lx;
                    nv[u] = min(VW, sx - lx);
#pragma unroll
                    for (int c = 0; c < NC; ++c) v[u][c] = *(const V*)(fg + c * a.ncell + gi);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (li[u] >= 0) {
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        const R* e = (const R*)&v[u][c];
#pragma unroll
                        for (int k = 0; k < VW; ++k)
                            if (k < nv[u]) fld[c * nsl + li[u] + k] = e[k];
                    }
                }
        }
    } else {
        // 4-byte / 8-byte loads, four in flight per thread before their stores
        const int sx = ext[0] + P - 1, sy = ext[1] + P - 1, sz = ext[2] + P - 1;
        const int n = sx * sy * sz;
        constexpr int U = 4;
        for (int i0 = 0; i0 < n; i0 += U * blockDim.x) {
            R v[U][NC];
            int li[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * blockDim.x + threadIdx.x;
                li[u] = -1;
                if (i < n) {
                    const int lx = i % sx, ly = (i / sx) % sy, lz = i / (sx * sy);
                    int gx = T0[0] + lx, gy = T0[1] + ly, gz = T0[2] + lz;
                    if (gx >= g.K[0]) gx -= g.K[0];
                    if (gy >= g.K[1]) gy -= g.K[1];
                    if (gz >= g.K[2]) gz -= g.K[2];
                    const size_t gi = ((size_t)gz * g.K[1] + gy) * g.K[0] + gx;
                    li[u] = lz * plane + ly * a.pitch_x + lx;
#pragma unroll
                    for (int c = 0; c < NC; ++c) v[u][c] = fg[c * a.ncell + gi];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (li[u] >= 0) {
#pragma unroll
                    for (int c = 0; c < NC; ++c) fld[c * nsl + li[u]] = v[u][c];
                }
        }
    }

    double gE = 1.0, Q = 0.0;
    if (MODE == GATHER_ADJOINT) {
        gE = *a.grad_energy;
        Q = a.eterms[4];
    }

    // Lane assignment.  A wavefront's LDS reads address the same offset from
    // 64 different stencil starts; when the starts fall in distinct LDS banks
    // the reads are conflict-free.  Each chunk of the tile's charges is
    // counting-sorted by the bank of its stencil start, and sorted position k
    // goes to wavefront k % nw, lane k / nw: each wavefront gets every nw-th
    // key in sorted order, i.e. starts spread over all banks.  In the mixed
    // form the records and caller indices move through LDS in the sort, and
    // the next chunk's are loaded while this one is summed; the FP64 form
    // sorts positions only and reads the records again (its LDS goes to the
    // staged field).
    constexpr bool MOVE = sizeof(R) == 4;
    RT* srec = (RT*)(smem_raw + a.sort_off);  // [blockDim] records in sorted order (mixed)
    int* sperm = MOVE ? (int*)(srec + blockDim.x) : (int*)(smem_raw + a.sort_off);  // [blockDim] caller
                                                                                   // indices / positions
    int* khist = sperm + blockDim.x;           // [64] bank histogram, then its prefix
    constexpr int KEYS = sizeof(R) == 4 ? 64 : 32;  // banks spanned by distinct starts

    // ad self-force coefficients, loaded once; uniform, so they are kept in
    // scalar registers
    R sf1[3] = {R(0), R(0), R(0)}, sf2[3] = {R(0), R(0), R(0)};
    const bool self_force = MODE == GATHER_AD && a.sfc != nullptr;
    if (self_force) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            sf1[d] = uniform((R)a.sfc[d]);
            sf2[d] = uniform((R)a.sfc[3 + d]);
        }
    }

    int l[3] = {0, 0, 0};
    R w[3][P], dw[3][P];
    for (int c0 = first; c0 < last; c0 += blockDim.x) {
        const int cnt = min((int)blockDim.x, last - c0);
        const bool have = (int)threadIdx.x < cnt;
        int key = 0;
        if (have) {
            const R tt[3] = {pr.x, pr.y, pr.z};
            int s3[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                R f;
                decode_local<R>(tt[d], ext[d], s3[d], f);
            }
            key = (s3[2] * plane + s3[1] * a.pitch_x + s3[0]) & (KEYS - 1);
        }
        if (threadIdx.x < 64) khist[threadIdx.x] = 0;
        // also completes the staging (first chunk) and the previous chunk's
        // reads of the sort buffers
        __syncthreads();
        const int rank = have ? atomicAdd(&khist[key], 1) : 0;
        __syncthreads();
        if (threadIdx.x < 64) {
            const int v = khist[threadIdx.x];
            khist[threadIdx.x] = wave_inclusive_scan(v) - v;
        }
        __syncthreads();
        if (have) {
            const int dst = khist[key] + rank;
            if constexpr (MOVE) {
                srec[dst] = pr;
                sperm[dst] = pm;
            } else {
                sperm[dst] = c0 + (int)threadIdx.x;
            }
        }
        const int nx = c0 + (int)blockDim.x + (int)threadIdx.x;
        if (nx < last) {
            pr = rec[nx];
            if constexpr (MOVE) pm = a.perm[nx];
        }
        __syncthreads();
        const int nw = (cnt + 63) >> 6;
        const int k = (threadIdx.x & 63) * nw + (int)(threadIdx.x >> 6);
        if ((int)(threadIdx.x >> 6) < nw && k < cnt) {
            RT r;
            int iu;
            if constexpr (MOVE) {
                r = srec[k];
                iu = sperm[k];
            } else {
                const int pc = sperm[k];
                r = rec[pc];
                iu = a.perm[pc];
            }
            {
                const R tt[3] = {r.x, r.y, r.z};
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    R f;
                    decode_local<R>(tt[d], ext[d], l[d], f);  // own charge: start in [0, ext)
                    stencil_weights<P, R, DERIV, TAB>(f, g, w[d], dw[d]);
                }
            }
            const R* base = fld + l[2] * plane + l[1] * a.pitch_x + l[0];
            R o0 = R(0), o1 = R(0), o2 = R(0), o3 = R(0);
            // z planes in a rolled loop: the plane's z coefficients are always
            // element 0 of the register arrays, which shift down one per plane
            // (no dynamic register indexing, P^2 loads in flight at most).
#pragma unroll 1
            for (int jz = 0; jz < P; ++jz) {
                R p0 = R(0), p1 = R(0), p2 = R(0);
                const R* pl0 = base + jz * plane;
#pragma unroll
                for (int jy = 0; jy < P; ++jy) {
                    const R* row = pl0 + jy * a.pitch_x;
                    if (MODE == GATHER_IK) {
                        R rx = R(0), ry = R(0), rz = R(0);
#pragma unroll
                        for (int jx = 0; jx < P; ++jx) {
                            rx += w[0][jx] * row[jx];
                            ry += w[0][jx] * row[nsl + jx];
                            rz += w[0][jx] * row[2 * nsl + jx];
                        }
                        p0 += w[1][jy] * rx;
                        p1 += w[1][jy] * ry;
                        p2 += w[1][jy] * rz;
                    } else {
                        R r0 = R(0), r1 = R(0);
#pragma unroll
                        for (int jx = 0; jx < P; ++jx) {
                            const R phi = row[jx];
                            r0 += w[0][jx] * phi;
                            r1 += dw[0][jx] * phi;
                        }
                        p0 += w[1][jy] * r1;   // -> d/dx
                        p1 += dw[1][jy] * r0;  // -> d/dy
                        p2 += w[1][jy] * r0;   // -> d/dz and the potential
                    }
                }
                const R wz = w[2][0], dwz = dw[2][0];
                if (MODE == GATHER_IK) {
                    o0 += wz * p0;
                    o1 += wz * p1;
                    o2 += wz * p2;
                } else {
                    o0 += wz * p0;
                    o1 += wz * p1;
                    o2 += dwz * p2;
                    o3 += wz * p2;
                }
#pragma unroll
                for (int j = 0; j < P - 1; ++j) {
                    w[2][j] = w[2][j + 1];
                    if (DERIV) dw[2][j] = dw[2][j + 1];
                }
            }
            TO* out = (TO*)a.out0;
            const R qv = r.w;
            if (MODE == GATHER_IK) {
                out[3 * (size_t)iu + 0] = (TO)(qv * o0);
                out[3 * (size_t)iu + 1] = (TO)(qv * o1);
                out[3 * (size_t)iu + 2] = (TO)(qv * o2);
            } else if (MODE == GATHER_AD) {
                R fo[3] = {-qv * o0 * (R)a.inv_h[0], -qv * o1 * (R)a.inv_h[1], -qv * o2 * (R)a.inv_h[2]};
                if (self_force) {
                    // self-force q^2 (c1_d sin(2 pi f_d) + c2_d sin(4 pi f_d)) with f_d the
                    // stencil fraction (re-read from the record); c1 carries the sign
                    // that turns sin(2 pi f) into sin(2 pi u) for odd orders
                    const R tt[3] = {r.x, r.y, r.z};
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        int sd;
                        R f;
                        decode_local<R>(tt[d], ext[d], sd, f);
                        fo[d] -= qv * qv * (sf1[d] * sin_turns(f) + sf2[d] * sin_turns(R(2) * f));
                    }
                }
                out[3 * (size_t)iu + 0] = (TO)fo[0];
                out[3 * (size_t)iu + 1] = (TO)fo[1];
                out[3 * (size_t)iu + 2] = (TO)fo[2];
            } else {
                const double qd = (double)qv;
                if (out) {
                    out[3 * (size_t)iu + 0] = (TO)(gE * qd * (double)o0 * a.inv_h[0]);
                    out[3 * (size_t)iu + 1] = (TO)(gE * qd * (double)o1 * a.inv_h[1]);
                    out[3 * (size_t)iu + 2] = (TO)(gE * qd * (double)o2 * a.inv_h[2]);
                }
                if (a.out1)
                    ((TO*)a.out1)[iu] = (TO)(gE * ((double)o3 - a.self_coef * qd - a.bg_coef * Q));
            }
        }
    }
}

template <int MODE, typename R, typename TO, bool TAB>
hipError_t dispatch_gather(int P, dim3 grid, dim3 block, size_t lds, hipStream_t st, const GatherArgs& a)
{
    switch (P) {
    case 2: k_gather<2, MODE, R, TO, TAB><<<grid, block, lds, st>>>(a); break;
    case 3: k_gather<3, MODE, R, TO, TAB><<<grid, block, lds, st>>>(a); break;
    case 4: k_gather<4, MODE, R, TO, TAB><<<grid, block, lds, st>>>(a); break;
    case 5: k_gather<5, MODE, R, TO, TAB><<<grid, block, lds, st>>>(a); break;
    case 6: k_gather<6, MODE, R, TO, TAB><<<grid, block, lds, st>>>(a); break;
    case 7: k_gather<7, MODE, R, TO, TAB><<<grid, block, lds, st>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int MODE, typename R, typename TO>
hipError_t dispatch_tab(const pppm_plan_s* pl, int P, dim3 grid, dim3 block, size_t lds, const GatherArgs& a)
{
    return pl->geo.wtab ? dispatch_gather<MODE, R, TO, true>(P, grid, block, lds, pl->stream, a)
                        : dispatch_gather<MODE, R, TO, false>(P, grid, block, lds, pl->stream, a);
}

template <int MODE>
hipError_t dispatch_types(const pppm_plan_s* pl, dim3 grid, dim3 block, size_t lds, const GatherArgs& a)
{
    const bool f32io = pl->p.io_dtype == PPPM_F32;
    const int P = pl->p.order;
    if (pl->mixed)
        return f32io ? dispatch_tab<MODE, float, float>(pl, P, grid, block, lds, a)
                     : dispatch_tab<MODE, float, double>(pl, P, grid, block, lds, a);
    return f32io ? dispatch_tab<MODE, double, float>(pl, P, grid, block, lds, a)
                 : dispatch_tab<MODE, double, double>(pl, P, grid, block, lds, a);
}

}  // namespace

// LDS of the staged field meshes (tile + upper halo), rounded up to 32 bytes
// (the alignment of the sorted records that follow).
size_t gather_field_lds_bytes(const MapGeo& g, int order, int ncomp, size_t elem_bytes)
{
    const size_t b = (size_t)ncomp * (g.B[0] + order - 1) * (g.B[1] + order - 1) * (g.B[2] + order - 1) * elem_bytes;
    return (b + 31) & ~(size_t)31;
}

// LDS of the lane-assignment buffers of a workgroup of `threads`: per thread
// a record (4 reals, mixed form only) and an index, and the 64-entry bank
// histogram.
static size_t gather_sort_lds_bytes(int threads, size_t elem_bytes)
{
    const size_t per = (elem_bytes == 4 ? 4 * elem_bytes : 0) + sizeof(int);
    return (size_t)threads * per + 64 * sizeof(int);
}

// Total LDS of a gather launch of `threads` threads: the staged meshes plus
// the lane-assignment buffers.
size_t gather_lds_bytes(const MapGeo& g, int order, int ncomp, size_t elem_bytes, int threads)
{
    return gather_field_lds_bytes(g, order, ncomp, elem_bytes) + gather_sort_lds_bytes(threads, elem_bytes);
}

hipError_t launch_gather(pppm_plan_s* pl, int mode, void* out0, void* out1, const double* grad_energy)
{
    const LaunchCfg& c = (mode == GATHER_ADJOINT) ? pl->adjoint_cfg : pl->gather_cfg;
    const int P = pl->p.order;
    GatherArgs a{};
    a.g = pl->geo;
    a.offsets = pl->offsets;
    a.rec = pl->records;
    a.perm = pl->perm;
    a.ncell = pl->ncell;
    a.pitch_x = pl->geo.B[0] + P - 1;
    a.rows_y = pl->geo.B[1] + P - 1;
    for (int d = 0; d < 3; ++d) a.inv_h[d] = 1.0 / pl->geo.h[d];
    a.out0 = out0;
    a.out1 = out1;
    a.grad_energy = grad_energy;
    a.eterms = pl->eterms;
    a.sfc = pl->sfc;
    a.self_coef = 2.0 * pl->p.coulomb_c * pl->p.g_ewald / sqrt(M_PI);
    const double V = pl->p.box_len[0] * pl->p.box_len[1] * pl->p.box_len[2];
    a.bg_coef = pl->p.coulomb_c * M_PI / (V * pl->p.g_ewald * pl->p.g_ewald);
    const size_t rs = pl->rsize;
    // 16-byte staging needs every row start (a multiple of B_x, or 0 after
    // the wrap) and K_x to be multiples of the chunk width
    const int vw = 16 / (int)rs;
    a.vec_stage = (pl->geo.K[0] % vw == 0) && (pl->geo.B[0] % vw == 0);
    dim3 grid(pl->geo.ntiles), block(c.threads);
    const int nc = mode == GATHER_IK ? 3 : 1;
    a.sort_off = (int)gather_field_lds_bytes(pl->geo, P, nc, rs);
    const size_t lds = a.sort_off + gather_sort_lds_bytes(c.threads, rs);
    switch (mode) {
    case GATHER_IK:
        a.field = pl->field;
        return dispatch_types<GATHER_IK>(pl, grid, block, lds, a);
    case GATHER_AD:
        a.field = pl->field;
        return dispatch_types<GATHER_AD>(pl, grid, block, lds, a);
    default:
        // phi lives after the three field meshes for ik plans, first for ad plans
        a.field = (const char*)pl->field + (pl->p.diff == PPPM_DIFF_IK ? 3 * pl->ncell * rs : 0);
        return dispatch_types<GATHER_ADJOINT>(pl, grid, block, lds, a);
    }
}

}  // namespace pppm
