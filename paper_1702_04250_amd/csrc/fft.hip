// The Poisson step (Equation 2; Section 3.2) as five passes over the mesh
// for meshes whose sizes are powers of two (8 .. 1024 in the mixed form,
// 8 .. 256 in FP64) or, in the mixed form, 2^a m with m in {3, 5, 7, 9}
// (12 .. 448; K_x / 2 from the same list); other sizes use rocFFT
// (plan.hip).
//
//   1. x, forward: each mesh row of K_x reals is packed as K_x / 2 complex
//      values (even points real, odd points imaginary), transformed, and
//      split into the K_x / 2 + 1 coefficients of the real transform.
//   2. y, forward: columns along y of the half spectrum, in place.
//   3. z: columns along z are transformed forward, multiplied by the
//      influence function (ik: and by -i kappa_d, three outputs), the FP64
//      energy partial sums taken, and transformed back along z.
//   4. y, inverse, per output mesh, in place.
//   5. x, inverse: each row's K_x / 2 + 1 coefficients are folded into
//      K_x / 2 complex values, transformed back and unpacked into K_x reals;
//      one extra block of this pass takes the final FP64 energy sums.
// In the mixed form, planes of at most XY_MAX complex values run passes 1+2
// and 4+5 fused, one z plane per block (k_fft_xy_fwd, k_fft_yx_inv).
//
// Each pass reads and writes the mesh once.  Conventions are those of the
// library's transforms: forward sum_m rho_m exp(-i k.m h), inverse
// unnormalised with exp(+i k.m h).  The half spectrum is stored
// [K_z][K_y][nxp] with the K_x/2 + 1 coefficients of a row padded to a
// 128-byte pitch, so that the column passes read whole cache lines; the
// influence function is read from its stored octant k_y, k_z >= 0.
//
// Every transform of length N = N1 N2 is done in two register stages with
// one exchange through LDS (the four-step split of the index,
// n = t + N2 j, k = k1 + N1 k2):
//   stage A: for each t, a length-N1 transform over j in registers, times
//            the twiddle W_N^(t k1);
//   stage B: for each k1, a length-N2 transform over t in registers.
// The short transforms are unrolled mixed-radix (2, 3, 5, 7) recursions
// whose roots are compile-time constants; the twiddles W_N come from
// per-axis tables computed in FP64 at plan creation.
#include "device_common.h"
#include "energy_sum.h"

namespace pppm {

namespace {

constexpr int FFT_THREADS = 256;

// complex value of the spectra (same layout as float2 / double2)
template <typename R> struct alignas(2 * sizeof(R)) Cplx {
    R x, y;
};

template <typename R> __device__ __forceinline__ Cplx<R> cmul(Cplx<R> a, Cplx<R> b)
{
    return Cplx<R>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// ---- compile-time roots of unity -------------------------------------------

constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double x)
{
    double t = x, s = x;
    for (int n = 1; n < 14; ++n) {
        t *= -x * x / (double)((2 * n) * (2 * n + 1));
        s += t;
    }
    return s;
}
constexpr double taylor_cos(double x)
{
    double t = 1.0, s = 1.0;
    for (int n = 1; n < 14; ++n) {
        t *= -x * x / (double)((2 * n - 1) * (2 * n));
        s += t;
    }
    return s;
}
// cos and sin of 2 pi k / L: the angle is reduced to its quadrant exactly
// (integer arithmetic), then the series run on [0, pi/2).
constexpr double root_cos(int k, int L)
{
    const int r = ((k % L) + L) % L;
    const int q = (4 * r) / L;
    const double x = 2.0 * kPi * (double)(4 * r - q * L) / (4.0 * (double)L);
    return q == 0 ? taylor_cos(x) : q == 1 ? -taylor_sin(x) : q == 2 ? -taylor_cos(x) : taylor_sin(x);
}
constexpr double root_sin(int k, int L)
{
    const int r = ((k % L) + L) % L;
    const int q = (4 * r) / L;
    const double x = 2.0 * kPi * (double)(4 * r - q * L) / (4.0 * (double)L);
    return q == 0 ? taylor_sin(x) : q == 1 ? taylor_cos(x) : q == 2 ? -taylor_sin(x) : -taylor_cos(x);
}

// Smallest prime factor of L among 2, 3, 5, 7 (L is 7-smooth).
constexpr int small_factor(int L) { return L % 2 == 0 ? 2 : L % 3 == 0 ? 3 : L % 5 == 0 ? 5 : 7; }

// a * exp(-+2 pi i n / L) (INV: +) with a compile-time root; the trivial
// roots cost no multiply
template <bool INV, typename R>
__device__ __forceinline__ Cplx<R> rot(Cplx<R> a, int n, int L)
{
    const int r = n % L;
    if (r == 0) return a;
    if (4 * r == L) return INV ? Cplx<R>{-a.y, a.x} : Cplx<R>{a.y, -a.x};  // -+i
    if (2 * r == L) return Cplx<R>{-a.x, -a.y};
    if (4 * r == 3 * L) return INV ? Cplx<R>{a.y, -a.x} : Cplx<R>{-a.y, a.x};  // +-i
    const R c = (R)root_cos(r, L);
    const R sn = INV ? (R)root_sin(r, L) : (R)-root_sin(r, L);
    return Cplx<R>{c * a.x - sn * a.y, c * a.y + sn * a.x};
}

// v <- DFT_L(v), v[k] = sum_j v[j] exp(-+2 pi i j k / L) (INV: +), L
// 7-smooth up to 32, unrolled: decimation in time by the smallest prime
// factor p of L (p sub-transforms of the points j = i p + s, then p-point
// butterflies), all roots compile-time constants.
template <int L, bool INV, typename R> struct Dft {
    __device__ __forceinline__ static void run(Cplx<R>* v)
    {
        constexpr int p = small_factor(L), M = L / p;
        if constexpr (p == 2) {
            // radix 2 on two flat arrays (keeps long transforms in registers)
            Cplx<R> e[M], o[M];
#pragma unroll
            for (int i = 0; i < M; ++i) {
                e[i] = v[2 * i];
                o[i] = v[2 * i + 1];
            }
            Dft<M, INV, R>::run(e);
            Dft<M, INV, R>::run(o);
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const Cplx<R> t = rot<INV, R>(o[k], k, L);
                v[k] = Cplx<R>{e[k].x + t.x, e[k].y + t.y};
                v[k + M] = Cplx<R>{e[k].x - t.x, e[k].y - t.y};
            }
            return;
        }
        Cplx<R> sub[p][M];
#pragma unroll
        for (int j = 0; j < p; ++j)
#pragma unroll
            for (int i = 0; i < M; ++i) sub[j][i] = v[i * p + j];
#pragma unroll
        for (int j = 0; j < p; ++j) Dft<M, INV, R>::run(sub[j]);
#pragma unroll
        for (int k = 0; k < M; ++k) {
            Cplx<R> t[p];
#pragma unroll
            for (int j = 0; j < p; ++j) t[j] = rot<INV, R>(sub[j][k], j * k, L);
#pragma unroll
            for (int q = 0; q < p; ++q) {
                Cplx<R> acc = t[0];
#pragma unroll
                for (int j = 1; j < p; ++j) {
                    const Cplx<R> u = rot<INV, R>(t[j], j * q, p);
                    acc = Cplx<R>{acc.x + u.x, acc.y + u.y};
                }
                v[k + q * M] = acc;
            }
        }
    }
};
template <bool INV, typename R> struct Dft<1, INV, R> {
    __device__ __forceinline__ static void run(Cplx<R>*) {}
};

// Split of N into N1 N2: N1 the smallest divisor with N1^2 >= N.
constexpr int split_n1(int N)
{
    for (int d = 1; d < N; ++d)
        if (N % d == 0 && d * d >= N) return d;
    return N;
}
template <int N> struct Split {
    static constexpr int N1 = split_n1(N);
    static constexpr int N2 = N / N1;
};

// Stage A of one task: v[j] holds element t + N2 j of sequence m; its
// length-N1 transform times W_N^(t k1) goes to ex.
template <int N1, int N2, bool INV, typename R>
__device__ __forceinline__ void stage_a(Cplx<R>* v, int t, int m, int lm, Cplx<R>* ex, const Cplx<R>* tw,
                                        int tstride)
{
    Dft<N1, INV, R>::run(v);
#pragma unroll
    for (int k1 = 1; k1 < N1; ++k1) {
        Cplx<R> w = tw[t * k1 * tstride];  // t k1 < N
        if (INV) w.y = -w.y;
        if (t != 0) v[k1] = cmul(v[k1], w);
    }
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) ex[((k1 * N2 + t) << lm) + m] = v[k1];
}

// Stage B of one task: v[k2] becomes coefficient k1 + N1 k2 of sequence m.
template <int N1, int N2, bool INV, typename R>
__device__ __forceinline__ void stage_b(Cplx<R>* v, int k1, int m, int lm, const Cplx<R>* ex)
{
#pragma unroll
    for (int t = 0; t < N2; ++t) v[t] = ex[((k1 * N2 + t) << lm) + m];
    Dft<N2, INV, R>::run(v);
}

// Transforms M sequences of length N (M a power of two).  ld(n, m) gives
// element n of sequence m, st(k, m, v) takes coefficient k; ex is an LDS
// buffer of N * M values; tw the LDS twiddle table with W_N^i at
// tw[i * tstride].  Every thread of the block must call it; it ends with a
// barrier.  Tasks map m fastest so that the lanes of a wavefront touch
// consecutive sequences.
template <int N, bool INV, typename R, typename Ld, typename St>
__device__ __forceinline__ void fft2(int M, Ld ld, St st, Cplx<R>* ex, const Cplx<R>* tw, int tstride)
{
    using C = Cplx<R>;
    constexpr int N1 = Split<N>::N1, N2 = Split<N>::N2;
    const int lm = __ffs(M) - 1;
    for (int task = threadIdx.x; task < N2 * M; task += blockDim.x) {
        const int m = task & (M - 1), t = task >> lm;
        C v[N1];
#pragma unroll
        for (int j = 0; j < N1; ++j) v[j] = ld(t + N2 * j, m);
        stage_a<N1, N2, INV, R>(v, t, m, lm, ex, tw, tstride);
    }
    __syncthreads();
    for (int task = threadIdx.x; task < N1 * M; task += blockDim.x) {
        const int m = task & (M - 1), k1 = task >> lm;
        C v[N2];
        stage_b<N1, N2, INV, R>(v, k1, m, lm, ex);
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) st(k1 + N1 * k2, m, v[k2]);
    }
    __syncthreads();
}

template <typename C> __device__ __forceinline__ void load_table(C* tw, const C* __restrict__ g, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) tw[i] = g[i];
}

// Element-wise copy of `total` items, dst(i) = src(i), with up to STAGE
// loads of each thread in flight before the first store.
constexpr int STAGE = 8;
template <typename T, typename Ld, typename St>
__device__ __forceinline__ void staged_copy(int total, Ld ld, St st)
{
    const int nt = blockDim.x;
    for (int i0 = threadIdx.x; i0 < total; i0 += STAGE * nt) {
        T v[STAGE];
#pragma unroll
        for (int u = 0; u < STAGE; ++u) {
            const int i = i0 + u * nt;
            if (i < total) v[u] = ld(i);
        }
#pragma unroll
        for (int u = 0; u < STAGE; ++u) {
            const int i = i0 + u * nt;
            if (i < total) st(i, v[u]);
        }
    }
}

struct FftGeo {
    int K[3];
    int nxh;            // K_x / 2 + 1 coefficients per row
    int nxp;            // row pitch of the spectra, nxh rounded up to 128 bytes
    double len[3];
    long long slot;     // elements per spectrum, K_z K_y nxp
};

// Pass 1.  `rows` rows of the real mesh per block (K_x = 2 NC points each)
// to rows of the half spectrum.  With z_n = x_2n + i x_2n+1 and Z its
// transform of length NC:
//   X_k = (Z_k + conj Z_{NC-k}) / 2 + W^k (Z_k - conj Z_{NC-k}) / 2i,
// W = exp(-2 pi i / K_x).  The rows are staged in LDS transposed, [n][m]
// with an odd pitch rows + 1, so that both the staging and the transform
// access LDS without bank conflicts.
template <typename R, int NC>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_x_fwd(const R* __restrict__ in, Cplx<R>* __restrict__ out,
                                                           int nxp, int nrows, int rows,
                                                           const Cplx<R>* __restrict__ twg)
{
    using C = Cplx<R>;
    constexpr int Kx = 2 * NC, nxh = NC + 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int P = rows + 1;
    C* tw = (C*)smem_raw;
    C* s = tw + Kx;        // [NC][P]
    C* ex = s + NC * P;    // [NC * rows]
    load_table(tw, twg, Kx);
    const int r0 = blockIdx.x * rows;
    const int nr = min(rows, nrows - r0);
    const C* src = (const C*)(in + (size_t)r0 * Kx);
    staged_copy<C>(
        rows * NC, [&](int i) { return (i < nr * NC) ? src[i] : C{R(0), R(0)}; },
        [&](int i, C v) {
            const int m = i / NC, n = i - m * NC;
            s[n * P + m] = v;
        });
    __syncthreads();
    fft2<NC, false, R>(
        rows, [&](int n, int m) { return s[n * P + m]; }, [&](int k, int m, C v) { s[k * P + m] = v; }, ex, tw, 2);
    for (int i = threadIdx.x; i < nr * nxh; i += blockDim.x) {
        const int m = i / nxh, k = i - m * nxh;
        const C za = s[(k == NC ? 0 : k) * P + m];
        const C zb = s[(k == 0 ? 0 : NC - k) * P + m];
        const C fe = C{R(0.5) * (za.x + zb.x), R(0.5) * (za.y - zb.y)};
        const C fo = C{R(0.5) * (za.y + zb.y), R(-0.5) * (za.x - zb.x)};
        const C wf = cmul(tw[k], fo);
        out[(size_t)(r0 + m) * nxp + k] = C{fe.x + wf.x, fe.y + wf.y};
    }
}

// Passes 2 and 4.  Columns along y of one z plane, xc adjacent x per block,
// in place (each block owns its columns); blockIdx.y selects the mesh of a
// batch (comp_stride apart).  Loads come straight from the mesh into
// registers and results go straight back.
template <typename R, int KY, bool INV>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_y(Cplx<R>* __restrict__ data, int nxh, int nxp, int xc, int nchunk,
                                                       long long comp_stride, const Cplx<R>* __restrict__ twg)
{
    using C = Cplx<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* tw = (C*)smem_raw;
    C* ex = tw + KY;
    load_table(tw, twg, KY);
    __syncthreads();
    const int z = blockIdx.x / nchunk, ch = blockIdx.x - z * nchunk;
    const int x0 = ch * xc, nx = min(xc, nxh - x0);
    C* d = data + blockIdx.y * comp_stride + (size_t)z * KY * nxp + x0;
    fft2<KY, INV, R>(
        xc, [&](int n, int m) { return (m < nx) ? d[(size_t)n * nxp + m] : C{R(0), R(0)}; },
        [&](int k, int m, C v) {
            if (m < nx) d[(size_t)k * nxp + m] = v;
        },
        ex, tw, 1);
}

__device__ __forceinline__ int fft_index(int i, int K) { return (2 * i < K) ? i : i - K; }

// Pass 3.  MODE 0 (ik): spec_d = z-inverse of -i kappa_d G' rho_hat, d = 0..2,
// kappa = 0 on the Nyquist planes; MODE 1 (ad): spec_0 = z-inverse of
// G' rho_hat; MODE 2: the potential alone into spec_0 (no energy).  Energy
// partial per block: sum w_k G' |rho_hat|^2, w_k = 1/2 on the x = 0 and
// x Nyquist planes (their Hermitian partners are not stored) and 1 elsewhere.
//
// The forward transform uses the split (N1, N2) and the inverse the split
// (N2, N1): stage B of the forward leaves each task with the coefficients
// k1 + N1 k2, k2 < N2, which are exactly the elements stage A of the
// inverse takes, so the multiply happens in registers between the two
// transforms with no LDS pass of its own.  One task per thread (the host
// keeps N1 * xc <= FFT_THREADS).
template <typename R, int KZ, int MODE>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_z_solve(const Cplx<R>* __restrict__ A, Cplx<R>* __restrict__ spec,
                                                             const double* __restrict__ G,
                                                             double* __restrict__ epart, FftGeo fg, int xc, int nchunk,
                                                             const Cplx<R>* __restrict__ twg)
{
    using C = Cplx<R>;
    constexpr int N1 = Split<KZ>::N1, N2 = Split<KZ>::N2;
    constexpr int NOUT = (MODE == 0) ? 3 : 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[FFT_THREADS / 64];
    const int Ky = fg.K[1], nxh = fg.nxh;
    const int cells = KZ * xc;
    C* tw = (C*)smem_raw;
    C* ex = tw + KZ;  // NOUT exchange buffers of `cells` values
    load_table(tw, twg, KZ);
    const int y = blockIdx.x / nchunk, ch = blockIdx.x - y * nchunk;
    const int x0 = ch * xc, nx = min(xc, nxh - x0);
    const size_t plane = (size_t)Ky * fg.nxp;
    const C* a = A + (size_t)y * fg.nxp + x0;
    const int lx = __ffs(xc) - 1;  // xc is a power of two
    // the thread's task between the transforms: sequence m, coefficients
    // k1 + N1 k2; its influence-function values (G octant: z <= K_z / 2,
    // y <= K_y / 2) are loaded first so that their latency overlaps the
    // forward transform
    const bool mid = (int)threadIdx.x < N1 * xc;
    const int mk1 = threadIdx.x >> lx, mm = threadIdx.x & (xc - 1);
    const bool live = mid && mm < nx;
    const int gny = Ky / 2 + 1;
    const int gy = min(y, Ky - y);
    double gk[N2];
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
        const int n = mk1 + N1 * k2;
        gk[k2] = live ? G[((size_t)min(n, KZ - n) * gny + gy) * nxh + x0 + mm] : 0.0;
    }
    __syncthreads();  // twiddle table
    // forward, stage A: global -> registers -> ex
    for (int task = threadIdx.x; task < N2 * xc; task += blockDim.x) {
        const int m = task & (xc - 1), t = task >> lx;
        C v[N1];
#pragma unroll
        for (int j = 0; j < N1; ++j) v[j] = (m < nx) ? a[(t + N2 * j) * plane + m] : C{R(0), R(0)};
        stage_a<N1, N2, false, R>(v, t, m, lx, ex, tw, 1);
    }
    __syncthreads();
    // forward, stage B, and the k-space multiply in registers
    C f[N2];
    double e = 0.0;
    if (mid) {
        stage_b<N1, N2, false, R>(f, mk1, mm, lx, ex);
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) {
            const double rx = (double)f[k2].x, ry = (double)f[k2].y;
            if (MODE != 2 && live) {
                const int ix = x0 + mm;
                const bool edge = (ix == 0) || (2 * ix == fg.K[0]);
                e += (edge ? 0.5 : 1.0) * gk[k2] * (rx * rx + ry * ry);
            }
            f[k2] = C{(R)(gk[k2] * rx), (R)(gk[k2] * ry)};  // G' rho_hat (0 off the mesh)
        }
    }
    __syncthreads();  // every task has read ex
    // inverse, stage A (split N2, N1) for each output
    if (mid) {
        const double two_pi = 2.0 * M_PI;
        for (int c = 0; c < NOUT; ++c) {
            C v[N2];
#pragma unroll
            for (int k2 = 0; k2 < N2; ++k2) {
                if (MODE == 0) {
                    const int n = mk1 + N1 * k2, ix = x0 + mm;
                    double kap;
                    if (c == 0)
                        kap = (2 * ix == fg.K[0]) ? 0.0 : two_pi * (double)fft_index(ix, fg.K[0]) / fg.len[0];
                    else if (c == 1)
                        kap = (2 * y == Ky) ? 0.0 : two_pi * (double)fft_index(y, Ky) / fg.len[1];
                    else
                        kap = (2 * n == KZ) ? 0.0 : two_pi * (double)fft_index(n, KZ) / fg.len[2];
                    // -i kappa (re + i im) = kappa im - i kappa re
                    v[k2] = C{(R)(kap * (double)f[k2].y), (R)(-kap * (double)f[k2].x)};
                } else {
                    v[k2] = f[k2];
                }
            }
            stage_a<N2, N1, true, R>(v, mk1, mm, lx, ex + c * cells, tw, 1);
        }
    }
    __syncthreads();
    // inverse, stage B: ex -> registers -> global
    for (int c = 0; c < NOUT; ++c) {
        C* out = spec + (size_t)c * fg.slot + (size_t)y * fg.nxp + x0;
        for (int task = threadIdx.x; task < N2 * xc; task += blockDim.x) {
            const int m = task & (xc - 1), k1 = task >> lx;
            C v[N1];
            stage_b<N2, N1, true, R>(v, k1, m, lx, ex + c * cells);
            if (m < nx) {
#pragma unroll
                for (int k2 = 0; k2 < N1; ++k2) out[(size_t)(k1 + N2 * k2) * plane + m] = v[k2];
            }
        }
    }
    if (MODE != 2) {
        for (int d = 32; d > 0; d >>= 1) e += __shfl_down(e, d, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
            epart[blockIdx.x] = s;
        }
    }
}

// Pass 5.  Rows of the half spectrum back to real rows: with
//   Z'_k = (X_k + conj X_{NC-k}) + i W^-k (X_k - conj X_{NC-k}),
// the inverse transform of Z' (length NC) is x_2n + i x_2n+1.
template <typename R, int NC>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_x_inv(const Cplx<R>* __restrict__ spec, R* __restrict__ out,
                                                           int nxp, int nrows, int rows, long long spec_stride,
                                                           long long out_stride, const Cplx<R>* __restrict__ twg,
                                                           EnergySums es, int final_sums)
{
    // one extra column of blocks: its first block takes the final energy
    // sums (the z pass that wrote the k-space partials has completed) on a
    // CU of its own, beside the transform blocks
    if (final_sums && blockIdx.x == gridDim.x - 1) {
        if (blockIdx.y == 0) energy_final_block(es);
        return;
    }
    using C = Cplx<R>;
    constexpr int Kx = 2 * NC, nxh = NC + 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int P = rows + 1;
    C* tw = (C*)smem_raw;
    C* xs = tw + Kx;         // [rows][nxh]
    C* s = xs + rows * nxh;  // [NC][P]
    C* ex = s + NC * P;      // [NC * rows]
    load_table(tw, twg, Kx);
    const int r0 = blockIdx.x * rows;
    const int nr = min(rows, nrows - r0);
    const C* src = spec + blockIdx.y * spec_stride + (size_t)r0 * nxp;
    staged_copy<C>(
        rows * nxh,
        [&](int i) {
            const int m = i / nxh, k = i - m * nxh;
            return (m < nr) ? src[(size_t)m * nxp + k] : C{R(0), R(0)};
        },
        [&](int i, C v) { xs[i] = v; });
    __syncthreads();
    for (int i = threadIdx.x; i < rows * NC; i += blockDim.x) {
        const int k = i / rows, m = i - k * rows;
        const C xa = xs[m * nxh + k];
        const C xb = xs[m * nxh + NC - k];  // used conjugated
        const C sm = C{xa.x + xb.x, xa.y - xb.y};
        const C d = C{xa.x - xb.x, xa.y + xb.y};
        const C w = C{tw[k].x, -tw[k].y};  // W^-k
        const C dw = cmul(d, w);
        s[k * P + m] = C{sm.x - dw.y, sm.y + dw.x};
    }
    __syncthreads();
    fft2<NC, true, R>(
        rows, [&](int n, int m) { return s[n * P + m]; }, [&](int k, int m, C v) { s[k * P + m] = v; }, ex, tw, 2);
    C* dst = (C*)(out + blockIdx.y * out_stride + (size_t)r0 * Kx);
    for (int i = threadIdx.x; i < nr * NC; i += blockDim.x) {
        const int m = i / NC, n = i - m * NC;
        dst[i] = s[n * P + m];
    }
}

// Passes 1 and 2 fused (mixed form, planes that fit in LDS): one z plane per
// block.  The x = 0 and x = K_x/2 coefficients of a row are real, so they
// travel together as one complex column Q = X_0 + i X_{K_x/2}; the y
// transform then runs on K_x / 2 columns, and the two real columns are
// separated afterwards by the symmetry of the transform of a real sequence,
//   Y_0(k) = (Q(k) + conj Q(-k)) / 2,   Y_{K_x/2}(k) = (Q(k) - conj Q(-k)) / 2i.
//
// HALF: two blocks per plane, one for the even and one for the odd y
// coefficients (radix-2 split of the y transform by output index).  With
// H = K_y / 2 and rows r_m of the plane,
//   Y(2j)   = sum_{m<H} (r_m + r_{m+H}) W_H^{jm},
//   Y(2j+1) = sum_{m<H} (r_m - r_{m+H}) W_{K_y}^m W_H^{jm},
// and the x transform is linear, so each block sums or subtracts the row
// pairs as it loads them and transforms H rows and H-point columns.  Every
// block reads the whole plane; the pass then has twice as many blocks,
// which a mesh of fewer planes than twice the CU count needs to fill the
// chip.  In the odd half the partner of coefficient j in the symmetry above
// is H - 1 - j (index -(2j+1) = 2(H-1-j)+1 mod K_y), in the even half
// (H - j) mod H.
// Both forms run 1024-thread blocks: a split pass has one block per CU on
// the meshes that take it, and the pass is bound by the latency of its
// load, exchange and store phases, which more wavefronts per CU hide (on
// 128^3: 512-thread split blocks 35.8 us for the Poisson step, 1024-thread
// 31.7 us, 256-thread 48.5 us).
constexpr int XY_THREADS = 1024;
constexpr int XY_HALF_THREADS = 1024;

// Block b of a split pass over nb = 2 * planes blocks: blocks b and b + 8
// take the two halves of one plane, so both run on one XCD and its L2
// serves the second read of the plane.
__device__ __forceinline__ void plane_half(int b, int nb, int& plane, int& h)
{
    if (nb % (2 * NUM_XCD) == 0) {
        plane = (b / (2 * NUM_XCD)) * NUM_XCD + b % NUM_XCD;
        h = (b / NUM_XCD) & 1;
    } else {
        plane = b >> 1;
        h = b & 1;
    }
}

template <typename R, int NC, int KY, bool HALF>
__global__ __launch_bounds__(HALF ? XY_HALF_THREADS : XY_THREADS) void k_fft_xy_fwd(const R* __restrict__ in,
                                                                                    Cplx<R>* __restrict__ out,
                                                                                    int nxp,
                                                                                    const Cplx<R>* __restrict__ twg)
{
    using C = Cplx<R>;
    constexpr int Kx = 2 * NC, KR = HALF ? KY / 2 : KY, P = KR + 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* twx = (C*)smem_raw;
    C* twy = twx + Kx;
    C* s = twy + KY;      // [NC][P]: rows transposed, then the y exchange buffer
    C* q = s + NC * P;    // [NC * KR]: the x exchange buffer, then the plane [y][k]
    load_table(twx, twg, Kx + KY);  // the x and y tables are adjacent
    int plane = blockIdx.x, h = 0;
    if constexpr (HALF) plane_half(blockIdx.x, gridDim.x, plane, h);
    const C* src = (const C*)(in + (size_t)plane * KY * Kx);
    staged_copy<C>(
        KR * NC,
        [&](int i) {
            C v = src[i];
            if constexpr (HALF) {
                const C w = src[i + KR * NC];  // row m + K_y / 2
                v = h ? C{v.x - w.x, v.y - w.y} : C{v.x + w.x, v.y + w.y};
            }
            return v;
        },
        [&](int i, C v) {
            const int m = i / NC, n = i - m * NC;
            s[n * P + m] = v;
        });
    __syncthreads();
    fft2<NC, false, R>(
        KR, [&](int n, int m) { return s[n * P + m]; }, [&](int k, int m, C v) { s[k * P + m] = v; }, q, twx, 2);
    // split into the half spectrum of each row; column 0 carries X_0 + i X_NC
    for (int i = threadIdx.x; i < KR * NC; i += blockDim.x) {
        const int m = i / NC, k = i - m * NC;
        const C za = s[k * P + m];
        const C zb = s[(k == 0 ? 0 : NC - k) * P + m];
        C x;
        if (k == 0) {
            // X_0 = Re Z_0 + Im Z_0, X_NC = Re Z_0 - Im Z_0
            x = C{za.x + za.y, za.x - za.y};
        } else {
            const C fe = C{R(0.5) * (za.x + zb.x), R(0.5) * (za.y - zb.y)};
            const C fo = C{R(0.5) * (za.y + zb.y), R(-0.5) * (za.x - zb.x)};
            const C wf = cmul(twx[k], fo);
            x = C{fe.x + wf.x, fe.y + wf.y};
        }
        if (HALF && h) x = cmul(x, twy[m]);  // W_{K_y}^m
        q[m * NC + k] = x;
    }
    __syncthreads();
    fft2<KR, false, R>(
        NC, [&](int n, int m) { return q[n * NC + m]; }, [&](int k, int m, C v) { q[k * NC + m] = v; }, s, twy,
        HALF ? 2 : 1);
    C* dst = out + (size_t)plane * KY * nxp;
    for (int i = threadIdx.x; i < KR * (NC + 1); i += blockDim.x) {
        const int j = i / (NC + 1), k = i - j * (NC + 1);
        C v;
        if (k > 0 && k < NC) {
            v = q[j * NC + k];
        } else {
            const int jp = (HALF && h) ? KR - 1 - j : (KR - j) % KR;
            const C a = q[j * NC];
            const C b = q[jp * NC];  // the partner, used conjugated
            v = (k == 0) ? C{R(0.5) * (a.x + b.x), R(0.5) * (a.y - b.y)}
                         : C{R(0.5) * (a.y + b.y), R(-0.5) * (a.x - b.x)};
        }
        const int ky = HALF ? 2 * j + h : j;
        dst[(size_t)ky * nxp + k] = v;
    }
}

// Passes 4 and 5 fused, one z plane of one output mesh per block.  The
// x = 0 and x = K_x/2 columns are Hermitian in k_y, so their y transforms
// are real: they go through one complex column Q = X_0 + i X_{K_x/2} and come
// out as its real and imaginary parts.
//
// HALF: two blocks per plane, one for the even and one for the odd output
// rows (radix-2 split of the inverse y transform by output index).  With
// H = K_y / 2,
//   x(2j)   = sum_{k<H} (X(k) + X(k+H)) W_H^{-jk},
//   x(2j+1) = sum_{k<H} (X(k) - X(k+H)) W_{K_y}^{-k} W_H^{-jk};
// the even and odd samples of the real columns x = 0 and x = K_x/2 are real
// too, so the packed column goes through unchanged.
template <typename R, int NC, int KY, bool HALF>
__global__ __launch_bounds__(HALF ? XY_HALF_THREADS : XY_THREADS) void k_fft_yx_inv(
    const Cplx<R>* __restrict__ spec, R* __restrict__ out, int nxp, long long spec_stride, long long out_stride,
    const Cplx<R>* __restrict__ twg, EnergySums es, int final_sums)
{
    // one extra column of blocks: its first block takes the final energy sums
    if (final_sums && blockIdx.x == gridDim.x - 1) {
        if (blockIdx.y == 0) energy_final_block(es);
        return;
    }
    using C = Cplx<R>;
    constexpr int Kx = 2 * NC, KR = HALF ? KY / 2 : KY, P = KR + 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* twx = (C*)smem_raw;
    C* twy = twx + Kx;
    C* s = twy + KY;    // [NC][P]: the y exchange buffer, then the rows transposed
    C* q = s + NC * P;  // [KR][NC]: the plane, then the x exchange buffer
    load_table(twx, twg, Kx + KY);
    int plane = blockIdx.x, h = 0;
    if constexpr (HALF) plane_half(blockIdx.x, gridDim.x - (final_sums ? 1 : 0), plane, h);
    const C* src = spec + blockIdx.y * spec_stride + (size_t)plane * KY * nxp;
    // row ky of the plane, column 0 packed as X_0 + i X_NC
    auto packed = [&](int ky, int k) {
        C v = src[(size_t)ky * nxp + k];
        if (k == 0) {
            const C b = src[(size_t)ky * nxp + NC];
            v = C{v.x - b.y, v.y + b.x};
        }
        return v;
    };
    staged_copy<C>(
        KR * NC,
        [&](int i) {
            const int ky = i / NC, k = i - ky * NC;
            C v = packed(ky, k);
            if constexpr (HALF) {
                const C w = packed(ky + KR, k);
                if (h) {
                    const C t = twg[Kx + ky];  // W_{K_y}^{ky}, used conjugated
                    v = cmul(C{v.x - w.x, v.y - w.y}, C{t.x, -t.y});
                } else {
                    v = C{v.x + w.x, v.y + w.y};
                }
            }
            return v;
        },
        [&](int i, C v) { q[i] = v; });
    __syncthreads();
    fft2<KR, true, R>(
        NC, [&](int n, int m) { return q[n * NC + m]; }, [&](int k, int m, C v) { q[k * NC + m] = v; }, s, twy,
        HALF ? 2 : 1);
    // fold each row into NC complex values: Z'_k = (X_k + conj X_{NC-k}) + i W^-k (X_k - conj X_{NC-k})
    for (int i = threadIdx.x; i < KR * NC; i += blockDim.x) {
        const int m = i / NC, k = i - m * NC;  // k fastest: row reads of q are consecutive
        const C w0 = q[m * NC];  // x_0 + i x_NC, both real
        const C xa = (k == 0) ? C{w0.x, R(0)} : q[m * NC + k];
        const C xb = (k == 0) ? C{w0.y, R(0)} : q[m * NC + NC - k];
        const C sm = C{xa.x + xb.x, xa.y - xb.y};
        const C d = C{xa.x - xb.x, xa.y + xb.y};
        const C w = C{twx[k].x, -twx[k].y};  // W^-k
        const C dw = cmul(d, w);
        s[k * P + m] = C{sm.x - dw.y, sm.y + dw.x};
    }
    __syncthreads();
    fft2<NC, true, R>(
        KR, [&](int n, int m) { return s[n * P + m]; }, [&](int k, int m, C v) { s[k * P + m] = v; }, q, twx, 2);
    C* dst = (C*)(out + blockIdx.y * out_stride + (size_t)plane * KY * Kx);
    for (int i = threadIdx.x; i < KR * NC; i += blockDim.x) {
        const int m = i / NC, n = i - m * NC;
        const int y = HALF ? 2 * m + h : m;
        dst[y * NC + n] = s[n * P + m];
    }
}

// Twiddle tables of the three axes, tw_d[i] = exp(-2 pi i * i / K_d), in FP64
// and rounded once to R.
template <typename R>
__global__ void k_fft_twiddles(Cplx<R>* __restrict__ tw, int Kx, int Ky, int Kz)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int total = Kx + Ky + Kz;
    if (i >= total) return;
    const int K = (i < Kx) ? Kx : (i < Kx + Ky ? Ky : Kz);
    const int j = (i < Kx) ? i : (i < Kx + Ky ? i - Kx : i - Kx - Ky);
    const double t = 2.0 * (double)j / (double)K;
    tw[i] = Cplx<R>{(R)cospi(t), (R)(-sinpi(t))};
}

FftGeo make_fgeo(const pppm_plan_s* pl)
{
    FftGeo fg{};
    for (int d = 0; d < 3; ++d) {
        fg.K[d] = pl->geo.K[d];
        fg.len[d] = pl->p.box_len[d];
    }
    fg.nxh = fg.K[0] / 2 + 1;
    fg.nxp = pl->fft_pitch;
    fg.slot = pl->spec_len;
    return fg;
}

// ---- dispatch over the transform lengths ----

struct Ctx {
    pppm_plan_s* pl;
    FftGeo fg;
    int mode, nout;
    void* A;      // Cplx<R>[slot]: x-y transformed mesh charge
    void* spec;   // Cplx<R>[nout * slot]
    void* field;  // R[nout * ncell]
    const void* tw;
    EnergySums es;   // final energy sums, taken by the last pass
    int final_sums;  // 0 for the potential alone
};

// Transform lengths the kernels are built for: powers of two (FP64 up to
// 256), and in the mixed form 2^a m, m in {3, 5, 7, 9}, up to 448.  A mesh
// axis of K points takes the length K (y, z) or K / 2 (x).
#define PPPM_FFT_POW2(X) X(4) X(8) X(16) X(32) X(64) X(128) X(256)
#define PPPM_FFT_MIXED_ONLY(X)                                                                              \
    X(512) X(1024) X(6) X(12) X(24) X(48) X(96) X(192) X(384) X(10) X(20) X(40) X(80) X(160) X(320) X(14) \
        X(28) X(56) X(112) X(224) X(448) X(18) X(36) X(72) X(144) X(288)

template <typename R, template <typename, int> class Launch>
bool by_length(int N, const Ctx& c)
{
#define PPPM_CASE(n)          \
    case n:                   \
        Launch<R, n>::go(c); \
        return true;
#define PPPM_CASE_MIXED(n)                  \
    case n:                                 \
        if constexpr (sizeof(R) == 4) {     \
            Launch<R, n>::go(c);           \
            return true;                    \
        }                                   \
        return false;
    switch (N) {
        PPPM_FFT_POW2(PPPM_CASE)
        PPPM_FFT_MIXED_ONLY(PPPM_CASE_MIXED)
    default:
        return false;
    }
#undef PPPM_CASE
#undef PPPM_CASE_MIXED
}

bool fft_length_ok(int n, bool mixed)
{
#define PPPM_YES(n) \
    case n:         \
        return true;
#define PPPM_IF_MIXED(n) \
    case n:              \
        return mixed;
    switch (n) {
        PPPM_FFT_POW2(PPPM_YES)
        PPPM_FFT_MIXED_ONLY(PPPM_IF_MIXED)
    default:
        return false;
    }
#undef PPPM_YES
#undef PPPM_IF_MIXED
}

template <typename R, int NC> struct XFwd {
    static void go(const Ctx& c)
    {
        const int nrows = c.fg.K[1] * c.fg.K[2], rows = c.pl->fx_rows;
        const size_t lds = sizeof(Cplx<R>) * (2 * NC + (size_t)NC * (rows + 1) + (size_t)NC * rows);
        k_fft_x_fwd<R, NC><<<(nrows + rows - 1) / rows, FFT_THREADS, lds, c.pl->stream>>>(
            (const R*)c.pl->rho, (Cplx<R>*)c.A, c.fg.nxp, nrows, rows, (const Cplx<R>*)c.tw);
    }
};
template <typename R, int NC> struct XInv {
    static void go(const Ctx& c)
    {
        const int nrows = c.fg.K[1] * c.fg.K[2], rows = c.pl->fx_rows;
        const size_t lds =
            sizeof(Cplx<R>) * (2 * NC + (size_t)rows * (NC + 1) + (size_t)NC * (rows + 1) + (size_t)NC * rows);
        k_fft_x_inv<R, NC><<<dim3((nrows + rows - 1) / rows + c.final_sums, c.nout), FFT_THREADS, lds,
                             c.pl->stream>>>(
            (const Cplx<R>*)c.spec, (R*)c.field, c.fg.nxp, nrows, rows, c.fg.slot, c.pl->ncell, (const Cplx<R>*)c.tw,
            c.es, c.final_sums);
    }
};
template <typename R, int KY> struct YFwd {
    static void go(const Ctx& c)
    {
        const int xc = c.pl->fy_xc, nch = (c.fg.nxh + xc - 1) / xc;
        const size_t lds = sizeof(Cplx<R>) * (KY + (size_t)KY * xc);
        k_fft_y<R, KY, false><<<dim3(c.fg.K[2] * nch, 1), FFT_THREADS, lds, c.pl->stream>>>(
            (Cplx<R>*)c.A, c.fg.nxh, c.fg.nxp, xc, nch, 0, (const Cplx<R>*)c.tw + c.fg.K[0]);
    }
};
template <typename R, int KY> struct YInv {
    static void go(const Ctx& c)
    {
        const int xc = c.pl->fy_xc, nch = (c.fg.nxh + xc - 1) / xc;
        const size_t lds = sizeof(Cplx<R>) * (KY + (size_t)KY * xc);
        k_fft_y<R, KY, true><<<dim3(c.fg.K[2] * nch, c.nout), FFT_THREADS, lds, c.pl->stream>>>(
            (Cplx<R>*)c.spec, c.fg.nxh, c.fg.nxp, xc, nch, c.fg.slot, (const Cplx<R>*)c.tw + c.fg.K[0]);
    }
};
template <typename R, int KZ> struct ZSolve {
    static void go(const Ctx& c)
    {
        const int xc = c.pl->fz_xc, nch = (c.fg.nxh + xc - 1) / xc;
        const size_t lds = sizeof(Cplx<R>) * (KZ + (size_t)(c.mode == 0 ? 3 : 1) * KZ * xc);
        const dim3 grid(c.fg.K[1] * nch);
        const Cplx<R>* tw = (const Cplx<R>*)c.tw + c.fg.K[0] + c.fg.K[1];
        const Cplx<R>* A = (const Cplx<R>*)c.A;
        Cplx<R>* spec = (Cplx<R>*)c.spec;
        switch (c.mode) {
        case 0:
            k_fft_z_solve<R, KZ, 0><<<grid, FFT_THREADS, lds, c.pl->stream>>>(A, spec, c.pl->G, c.pl->epart, c.fg, xc,
                                                                             nch, tw);
            break;
        case 1:
            k_fft_z_solve<R, KZ, 1><<<grid, FFT_THREADS, lds, c.pl->stream>>>(A, spec, c.pl->G, c.pl->epart, c.fg, xc,
                                                                             nch, tw);
            break;
        default:
            k_fft_z_solve<R, KZ, 2><<<grid, FFT_THREADS, lds, c.pl->stream>>>(A, spec, c.pl->G, c.pl->epart, c.fg, xc,
                                                                             nch, tw);
            break;
        }
    }
};

// Fused x-y passes: planes of NC * KY <= XY_MAX complex values (two such
// buffers stay within the LDS of one block).
constexpr int XY_MAX = 8192;

// LDS of a fused pass transforming kr rows of a plane (kr = K_y, or K_y / 2
// when the plane is split over two blocks).
size_t xy_lds_bytes(int nc, int ky, int kr)
{
    return sizeof(Cplx<float>) * (2 * nc + ky + (size_t)nc * (kr + 1) + (size_t)nc * kr);
}

// A pass with fewer blocks (one per plane and output mesh) than two per CU
// of the chip runs split, two blocks per plane.
constexpr int XY_SPLIT_BELOW = 512;

template <int NC, int KY, bool HALF> void xy_run(const Ctx& c, bool inverse)
{
    const size_t lds = xy_lds_bytes(NC, KY, HALF ? KY / 2 : KY);
    const int threads = HALF ? XY_HALF_THREADS : XY_THREADS;
    const int nb = HALF ? 2 * c.fg.K[2] : c.fg.K[2];
    const Cplx<float>* tw = (const Cplx<float>*)c.tw;
    if (!inverse)
        k_fft_xy_fwd<float, NC, KY, HALF><<<nb, threads, lds, c.pl->stream>>>((const float*)c.pl->rho,
                                                                             (Cplx<float>*)c.A, c.fg.nxp, tw);
    else
        k_fft_yx_inv<float, NC, KY, HALF><<<dim3(nb + c.final_sums, c.nout), threads, lds, c.pl->stream>>>(
            (const Cplx<float>*)c.spec, (float*)c.field, c.fg.nxp, c.fg.slot, c.pl->ncell, tw, c.es, c.final_sums);
}

template <int NC, int KY> void xy_go(const Ctx& c, bool inverse)
{
    if constexpr (NC * KY <= XY_MAX) {
        if (c.fg.K[2] * (inverse ? c.nout : 1) < XY_SPLIT_BELOW)
            xy_run<NC, KY, true>(c, inverse);
        else
            xy_run<NC, KY, false>(c, inverse);
    }
}

template <int NC> bool xy_by_ky(int ky, const Ctx& c, bool inverse)
{
    switch (ky) {
    case 16: xy_go<NC, 16>(c, inverse); return true;
    case 32: xy_go<NC, 32>(c, inverse); return true;
    case 64: xy_go<NC, 64>(c, inverse); return true;
    case 128: xy_go<NC, 128>(c, inverse); return true;
    case 256: xy_go<NC, 256>(c, inverse); return true;
    case 512: xy_go<NC, 512>(c, inverse); return true;
    default: return false;
    }
}

bool xy_launch(const Ctx& c, bool inverse)
{
    const int nc = c.fg.K[0] / 2, ky = c.fg.K[1];
    switch (nc) {
    case 16: return xy_by_ky<16>(ky, c, inverse);
    case 32: return xy_by_ky<32>(ky, c, inverse);
    case 64: return xy_by_ky<64>(ky, c, inverse);
    case 128: return xy_by_ky<128>(ky, c, inverse);
    case 256: return xy_by_ky<256>(ky, c, inverse);
    case 512: return xy_by_ky<512>(ky, c, inverse);
    default: return false;
    }
}

// mode: 0 ik forward (three fields), 1 ad forward (potential), 2 potential
// alone (into spectrum / mesh slot `slot`).
template <typename R>
hipError_t run_own_poisson(pppm_plan_s* pl, int mode, int slot, double* energy_out)
{
    if (mode != 2) pl->epart_blocks = pl->fz_blocks;
    Ctx c{};
    c.es = energy_sums(pl, energy_out);
    c.final_sums = (mode != 2);
    c.pl = pl;
    c.fg = make_fgeo(pl);
    c.mode = mode;
    c.nout = (mode == 0) ? 3 : 1;
    c.A = pl->rho_hat;
    c.spec = (Cplx<R>*)pl->spec + (size_t)slot * pl->spec_len;
    c.field = (R*)pl->field + (size_t)slot * pl->ncell;
    c.tw = pl->fft_tw;
    const int Nc = c.fg.K[0] / 2;
    // every length was checked at plan creation (own_fft_supported,
    // own_fft_shapes decides fft_xy)
    const bool xy = pl->fft_xy && sizeof(R) == 4;
    if (mode != 2) {
        if (xy) {
            if (!xy_launch(c, false)) return hipErrorInvalidValue;
        } else if (!by_length<R, XFwd>(Nc, c) || !by_length<R, YFwd>(c.fg.K[1], c)) {
            return hipErrorInvalidValue;
        }
    }
    if (!by_length<R, ZSolve>(c.fg.K[2], c)) return hipErrorInvalidValue;
    if (xy) {
        if (!xy_launch(c, true)) return hipErrorInvalidValue;
    } else if (!by_length<R, YInv>(c.fg.K[1], c) || !by_length<R, XInv>(Nc, c)) {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

bool own_fft_supported(const int K[3], bool mixed)
{
    // FP64 keeps to powers of two up to 256: register stages of at most 16 values
    return K[0] >= 8 && K[0] % 2 == 0 && fft_length_ok(K[0] / 2, mixed) && K[1] >= 8 && fft_length_ok(K[1], mixed) &&
           K[2] >= 8 && fft_length_ok(K[2], mixed);
}

// Launch shapes: about `target` complex values per block, fewer when that
// leaves too few blocks; x columns per block stay powers of two.
void own_fft_shapes(pppm_plan_s* pl)
{
    const int Kx = pl->geo.K[0], Ky = pl->geo.K[1], Kz = pl->geo.K[2];
    const int nxh = Kx / 2 + 1, Nc = Kx / 2;
    const int target = pl->mixed ? 2048 : 1024;
    const int nrows = Ky * Kz;
    // batch sizes (rows, x columns) are powers of two
    auto pow2_floor = [](int v) {
        int p = 1;
        while (2 * p <= v) p *= 2;
        return p;
    };
    int rows = pow2_floor(target / Nc > 0 ? target / Nc : 1);
    while (rows > 1 && (nrows + rows - 1) / rows < 512) rows /= 2;
    pl->fx_rows = rows;
    int xy = pow2_floor(target / Ky > 0 ? target / Ky : 1);
    if (xy > 16) xy = 16;
    while (xy > 4 && Kz * ((nxh + xy - 1) / xy) < 512) xy /= 2;
    pl->fy_xc = xy;
    int xz = pow2_floor(target / Kz > 0 ? target / Kz : 1);
    if (xz > 16) xz = 16;
    while (xz > 4 && Ky * ((nxh + xz - 1) / xz) < 512) xz /= 2;
    pl->fz_xc = xz;
    pl->fz_blocks = Ky * ((nxh + xz - 1) / xz);
    // x and y fused per plane: mixed form, powers of two 16 <= K_x / 2, K_y <= 512,
    // plane within XY_MAX
    const bool p2 = (Nc & (Nc - 1)) == 0 && (Ky & (Ky - 1)) == 0;
    pl->fft_xy = pl->mixed && p2 && Nc >= 16 && Ky >= 16 && Nc <= 512 && Ky <= 512 && Nc * Ky <= XY_MAX &&
                 xy_lds_bytes(Nc, Ky, Ky) + 1024 <= pl->lds_limit;
    const int per_line = 128 / (pl->mixed ? 8 : 16);
    pl->fft_pitch = (nxh + per_line - 1) / per_line * per_line;
    pl->spec_len = (int64_t)Kz * Ky * pl->fft_pitch;
}

// The z pass gives each thread at most one task between its transforms.
bool own_fft_shapes_ok(const pppm_plan_s* pl)
{
    return split_n1(pl->geo.K[2]) * pl->fz_xc <= FFT_THREADS;
}

size_t own_fft_lds_max(const pppm_plan_s* pl)
{
    const size_t csz = pl->mixed ? 8 : 16;
    const int Kx = pl->geo.K[0], Ky = pl->geo.K[1], Kz = pl->geo.K[2];
    const int Nc = Kx / 2;
    const size_t rows = pl->fx_rows;
    const size_t x_inv = csz * (Kx + rows * (Nc + 1) + (size_t)Nc * (rows + 1) + (size_t)Nc * rows);
    const size_t y = csz * (Ky + (size_t)Ky * pl->fy_xc);
    const size_t z = csz * (Kz + 3 * (size_t)Kz * pl->fz_xc);  // ik: three exchange buffers
    size_t m = x_inv > y ? x_inv : y;
    return m > z ? m : z;
}

hipError_t launch_own_fft_twiddles(pppm_plan_s* pl)
{
    const int total = pl->geo.K[0] + pl->geo.K[1] + pl->geo.K[2];
    const int blocks = (total + 255) / 256;
    if (pl->mixed)
        k_fft_twiddles<float><<<blocks, 256, 0, pl->stream>>>((Cplx<float>*)pl->fft_tw, pl->geo.K[0], pl->geo.K[1],
                                                              pl->geo.K[2]);
    else
        k_fft_twiddles<double><<<blocks, 256, 0, pl->stream>>>((Cplx<double>*)pl->fft_tw, pl->geo.K[0], pl->geo.K[1],
                                                               pl->geo.K[2]);
    return hipGetLastError();
}

hipError_t launch_own_poisson(pppm_plan_s* pl, bool phi_only, double* energy_out)
{
    const int mode = phi_only ? 2 : (pl->p.diff == PPPM_DIFF_IK ? 0 : 1);
    // the potential of an ik plan goes to the slot after its three fields
    const int slot = phi_only ? (pl->p.diff == PPPM_DIFF_IK ? 3 : 0) : 0;
    return pl->mixed ? run_own_poisson<float>(pl, mode, slot, energy_out)
                     : run_own_poisson<double>(pl, mode, slot, energy_out);
}

}  // namespace pppm
