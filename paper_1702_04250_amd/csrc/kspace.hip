// k-space part of the Poisson step (Equation 2; Section 3.2), around the
// rocFFT transforms: the influence function (built once per plan), the
// influence-function multiply with the ik derivative, and the FP64 energy
// reduction.
//
// Influence function (the paper leaves the Green function unspecified; this
// is the optimal one for order-P B-spline assignment, minimising the RMS
// force error): with U(k) = prod_d sinc(k_d h_d / 2)^P,
// R(k) = 4 pi exp(-k^2/4g^2) / k^2 and aliases k_m = k + 2 pi m / h, |m_d| <= 2,
//   ik: G = sum_m U^2(k_m) (k . k_m) R(k_m) / (|k|^2 [sum_m U^2(k_m)]^2)
//   ad: G = sum_m U^2(k_m) |k_m|^2 R(k_m) / ([sum_m U^2(k_m)] [sum_m |k_m|^2 U^2(k_m)])
// G(0) = 0.  The plan stores (C / V) G on the half spectrum of the real FFT,
// or, for the library's own transforms, on the octant k_y, k_z >= 0 of it
// only: G is even in each wavenumber component (the alias sums are
// symmetric), so G(k_x, -k_y, k_z) = G(k_x, k_y, k_z) and likewise in z.
#include "device_common.h"
#include "energy_sum.h"

namespace pppm {

namespace {

constexpr int ALIAS = 2;
constexpr int NA = 2 * ALIAS + 1;

struct KGeo {
    int K[3];
    int nxh;        // Kx / 2 + 1
    double len[3];
    double h[3];
    int gny, gnz;   // y and z extent of the stored G: K_y, K_z (full) or K/2 + 1 (one octant)
};

__device__ __forceinline__ void store_c(float2* p, double re, double im) { *p = make_float2((float)re, (float)im); }
__device__ __forceinline__ void store_c(double2* p, double re, double im) { *p = make_double2(re, im); }

// FFT-order wavenumber index: n in [-K/2, K/2)
__device__ __forceinline__ int fft_index(int i, int K) { return (2 * i < K) ? i : i - K; }

__global__ __launch_bounds__(KSPACE_THREADS) void k_influence(KGeo kg, long long nspec, int P, double g,
                                                               int diff, double scale, double* __restrict__ G)
{
    const long long idx = (long long)blockIdx.x * KSPACE_THREADS + threadIdx.x;
    if (idx >= nspec) return;
    const int ix = (int)(idx % kg.nxh);
    const int iy = (int)((idx / kg.nxh) % kg.gny);
    const int iz = (int)(idx / ((long long)kg.nxh * kg.gny));
    const int ii[3] = {ix, iy, iz};
    const double two_pi = 2.0 * M_PI;
    double kk[3];
    double qv[3][NA], u2[3][NA], ex[3][NA];
    for (int d = 0; d < 3; ++d) {
        kk[d] = two_pi * (double)fft_index(ii[d], kg.K[d]) / kg.len[d];
        for (int m = 0; m < NA; ++m) {
            const double q = kk[d] + two_pi * (double)(m - ALIAS) / kg.h[d];
            const double x = 0.5 * q * kg.h[d];
            const double s = (x == 0.0) ? 1.0 : sin(x) / x;
            double p = 1.0;
            for (int e = 0; e < 2 * P; ++e) p *= s;
            qv[d][m] = q;
            u2[d][m] = p;
            ex[d][m] = exp(-q * q / (4.0 * g * g));
        }
    }
    const double k2 = kk[0] * kk[0] + kk[1] * kk[1] + kk[2] * kk[2];
    double out = 0.0;
    if (k2 > 0.0) {
        double num = 0.0, sum_u2 = 0.0, sum_k2u2 = 0.0;
        for (int mz = 0; mz < NA; ++mz)
            for (int my = 0; my < NA; ++my)
                for (int mx = 0; mx < NA; ++mx) {
                    const double qx = qv[0][mx], qy = qv[1][my], qz = qv[2][mz];
                    const double u = u2[0][mx] * u2[1][my] * u2[2][mz];
                    const double q2 = qx * qx + qy * qy + qz * qz;
                    const double ref = (q2 > 0.0) ? 4.0 * M_PI * ex[0][mx] * ex[1][my] * ex[2][mz] / q2 : 0.0;
                    sum_u2 += u;
                    sum_k2u2 += q2 * u;
                    num += (diff == PPPM_DIFF_IK) ? u * (kk[0] * qx + kk[1] * qy + kk[2] * qz) * ref
                                                  : u * q2 * ref;
                }
        out = (diff == PPPM_DIFF_IK) ? num / (k2 * sum_u2 * sum_u2) : num / (sum_u2 * sum_k2u2);
    }
    G[idx] = scale * out;
}

// phi_hat = G' rho_hat; ik: E_hat_d = -i kappa_d G' rho_hat (kappa = 0 on the
// Nyquist planes); energy partial sums 1/2 sum w_k G' |rho_hat|^2 where w_k
// counts the Hermitian partner of each half-spectrum point.
template <typename C>
__global__ __launch_bounds__(KSPACE_THREADS) void k_solve(KGeo kg, long long nspec, int mode,
                                                           const C* __restrict__ rho_hat,
                                                           const double* __restrict__ G, C* __restrict__ spec,
                                                           double* __restrict__ epart)
{
    __shared__ double red[KSPACE_THREADS / 64];
    double e = 0.0;
    const double two_pi = 2.0 * M_PI;
    for (long long idx = (long long)blockIdx.x * KSPACE_THREADS + threadIdx.x; idx < nspec;
         idx += (long long)gridDim.x * KSPACE_THREADS) {
        const int ix = (int)(idx % kg.nxh);
        const double2 rh = make_double2((double)rho_hat[idx].x, (double)rho_hat[idx].y);
        const double gk = G[idx];
        const bool edge = (ix == 0) || (2 * ix == kg.K[0]);
        e += (edge ? 0.5 : 1.0) * gk * (rh.x * rh.x + rh.y * rh.y);
        const double re = gk * rh.x, im = gk * rh.y;
        if (mode == 1) {  // ad: potential only
            store_c(spec + idx, re, im);
        } else {
            const int iy = (int)((idx / kg.nxh) % kg.K[1]);
            const int iz = (int)(idx / ((long long)kg.nxh * kg.K[1]));
            const int ii[3] = {ix, iy, iz};
            for (int d = 0; d < 3; ++d) {
                const int n = (2 * ii[d] == kg.K[d]) ? 0 : fft_index(ii[d], kg.K[d]);
                const double kap = two_pi * (double)n / kg.len[d];
                // -i kappa (re + i im) = kappa im - i kappa re
                store_c(spec + d * nspec + idx, kap * im, -kap * re);
            }
        }
    }
    for (int d = 32; d > 0; d >>= 1) e += __shfl_down(e, d, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < KSPACE_THREADS / 64; ++w) s += red[w];
        epart[blockIdx.x] = s;
    }
}

// phi_hat only, into the slot after the ik field spectra (adjoint of ik plans).
template <typename C>
__global__ __launch_bounds__(KSPACE_THREADS) void k_phi_only(long long nspec, const C* __restrict__ rho_hat,
                                                              const double* __restrict__ G, C* __restrict__ out)
{
    for (long long idx = (long long)blockIdx.x * KSPACE_THREADS + threadIdx.x; idx < nspec;
         idx += (long long)gridDim.x * KSPACE_THREADS) {
        const double rx = (double)rho_hat[idx].x, ry = (double)rho_hat[idx].y;
        const double gk = G[idx];
        store_c(out + idx, gk * rx, gk * ry);
    }
}

// Deterministic final sums (energy_sum.h).
__global__ __launch_bounds__(1024) void k_energy_final(EnergySums es) { energy_final_block(es); }

// ad self-force coefficients.  A lone charge q at mesh coordinate u has the
// mesh energy (C q^2 / 2V) sum_k G sum_{a,b} U(k_a) U(k_b) cos(2 pi (a - b).u)
// (aliases k_a = k + 2 pi a / h, U = prod_d sinc(k_d h_d / 2)^P).  Its terms
// with a - b = +-e_d and +-2 e_d are the position-dependent energy
// q^2 [S1_d cos(2 pi u_d) + S2_d cos(4 pi u_d)] with
//   S1_d = sum_k G'(k) prod_{d' != d} [sum_a U_d'(a)^2] sum_a U_d(a) U_d(a + 1),
//   S2_d the same with U_d(a) U_d(a + 2),
// G' = (C/V) G the plan's influence function, |a_d| <= 2, the sum over the
// full spectrum (each half-spectrum point but the x = 0 and Nyquist planes
// stands for two).  Its negative gradient is the self-force.  One partial
// sum of (S1, S2) per block; the final kernel adds them in block order.
__global__ __launch_bounds__(KSPACE_THREADS) void k_self_force_partials(KGeo kg, long long nspec, int P,
                                                                         const double* __restrict__ G,
                                                                         double* __restrict__ part)
{
    __shared__ double red[6][KSPACE_THREADS / 64];
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const double two_pi = 2.0 * M_PI;
    for (long long idx = (long long)blockIdx.x * KSPACE_THREADS + threadIdx.x; idx < nspec;
         idx += (long long)gridDim.x * KSPACE_THREADS) {
        const int ix = (int)(idx % kg.nxh);
        const int iy = (int)((idx / kg.nxh) % kg.K[1]);
        const int iz = (int)(idx / ((long long)kg.nxh * kg.K[1]));
        const int ii[3] = {ix, iy, iz};
        double sq[3], b1[3], b2[3];
        for (int d = 0; d < 3; ++d) {
            const double kd = two_pi * (double)fft_index(ii[d], kg.K[d]) / kg.len[d];
            double u[NA];
            for (int m = 0; m < NA; ++m) {
                const double x = 0.5 * (kd + two_pi * (double)(m - ALIAS) / kg.h[d]) * kg.h[d];
                const double s = (x == 0.0) ? 1.0 : sin(x) / x;
                double p = 1.0;
                for (int e = 0; e < P; ++e) p *= s;
                u[m] = p;
            }
            sq[d] = b1[d] = b2[d] = 0.0;
            for (int m = 0; m < NA; ++m) sq[d] += u[m] * u[m];
            for (int m = 0; m + 1 < NA; ++m) b1[d] += u[m] * u[m + 1];
            for (int m = 0; m + 2 < NA; ++m) b2[d] += u[m] * u[m + 2];
        }
        const bool edge = (ix == 0) || (2 * ix == kg.K[0]);
        const int gy = (kg.gny == kg.K[1]) ? iy : min(iy, kg.K[1] - iy);
        const int gz = (kg.gnz == kg.K[2]) ? iz : min(iz, kg.K[2] - iz);
        const double wg = (edge ? 1.0 : 2.0) * G[((size_t)gz * kg.gny + gy) * kg.nxh + ix];
        acc[0] += wg * b1[0] * sq[1] * sq[2];
        acc[1] += wg * sq[0] * b1[1] * sq[2];
        acc[2] += wg * sq[0] * sq[1] * b1[2];
        acc[3] += wg * b2[0] * sq[1] * sq[2];
        acc[4] += wg * sq[0] * b2[1] * sq[2];
        acc[5] += wg * sq[0] * sq[1] * b2[2];
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int j = 0; j < 6; ++j) {
        double v = acc[j];
        for (int d = 32; d > 0; d >>= 1) v += __shfl_down(v, d, 64);
        if (lane == 0) red[j][wid] = v;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double v = 0.0;
        for (int w = 0; w < KSPACE_THREADS / 64; ++w) v += red[threadIdx.x][w];
        part[6 * (size_t)blockIdx.x + threadIdx.x] = v;
    }
}

// Coefficients of the self-force in terms of the stencil fraction f the
// gather holds: u = s + f + P/2 - 1 with s an integer, so sin(2 pi u) =
// (-1)^P sin(2 pi f) and sin(4 pi u) = sin(4 pi f).
// coef[d] = (-1)^P 2 pi S1_d / h_d, coef[3 + d] = 4 pi S2_d / h_d.
__global__ __launch_bounds__(64) void k_self_force_final(int nblocks, KGeo kg, int P, const double* __restrict__ part,
                                                         double* __restrict__ coef)
{
    const int j = threadIdx.x;
    if (j >= 6) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += part[6 * (size_t)b + j];
    const double odd = (P & 1) ? -1.0 : 1.0;
    coef[j] = (j < 3 ? odd * 2.0 * M_PI / kg.h[j] : 4.0 * M_PI / kg.h[j - 3]) * s;
}

KGeo make_kgeo(const pppm_plan_s* pl)
{
    KGeo kg{};
    for (int d = 0; d < 3; ++d) {
        kg.K[d] = pl->geo.K[d];
        kg.len[d] = pl->p.box_len[d];
        kg.h[d] = pl->geo.h[d];
    }
    kg.nxh = kg.K[0] / 2 + 1;
    kg.gny = pl->own_fft ? kg.K[1] / 2 + 1 : kg.K[1];
    kg.gnz = pl->own_fft ? kg.K[2] / 2 + 1 : kg.K[2];
    return kg;
}

}  // namespace

EnergySums energy_sums(const pppm_plan_s* pl, double* energy_out)
{
    const double V = pl->p.box_len[0] * pl->p.box_len[1] * pl->p.box_len[2];
    const double C = pl->p.coulomb_c, g = pl->p.g_ewald;
    EnergySums es{};
    es.ne = (int)pl->epart_blocks;
    es.epart = pl->epart;
    es.nq = (int)pl->qpart_blocks;
    es.qpart = pl->qpart;
    es.self_c = C * g / sqrt(M_PI);
    es.bg_c = C * M_PI / (2.0 * V * g * g);
    es.eterms = pl->eterms;
    es.energy_out = energy_out;
    return es;
}

int kspace_blocks(long long nspec)
{
    const long long b = (nspec + KSPACE_THREADS - 1) / KSPACE_THREADS;
    return (int)(b < 2048 ? (b < 1 ? 1 : b) : 2048);
}

hipError_t launch_self_force_coef(pppm_plan_s* pl)
{
    const KGeo kg = make_kgeo(pl);
    const int blocks = kspace_blocks(pl->nspec);
    k_self_force_partials<<<blocks, KSPACE_THREADS, 0, pl->stream>>>(kg, pl->nspec, pl->p.order, pl->G,
                                                                      pl->sfc + 6);
    k_self_force_final<<<1, 64, 0, pl->stream>>>(blocks, kg, pl->p.order, pl->sfc + 6, pl->sfc);
    return hipGetLastError();
}

hipError_t launch_influence(pppm_plan_s* pl)
{
    const KGeo kg = make_kgeo(pl);
    const double V = pl->p.box_len[0] * pl->p.box_len[1] * pl->p.box_len[2];
    const long long ng = (long long)kg.nxh * kg.gny * kg.gnz;
    const long long blocks = (ng + KSPACE_THREADS - 1) / KSPACE_THREADS;
    k_influence<<<(unsigned)blocks, KSPACE_THREADS, 0, pl->stream>>>(
        kg, ng, pl->p.order, pl->p.g_ewald, (int)pl->p.diff, pl->p.coulomb_c / V, pl->G);
    return hipGetLastError();
}

hipError_t launch_kspace(pppm_plan_s* pl, bool phi_only)
{
    const KGeo kg = make_kgeo(pl);
    const int blocks = kspace_blocks(pl->nspec);
    if (phi_only) {
        const size_t csz = pl->mixed ? sizeof(float2) : sizeof(double2);
        void* out = (char*)pl->spec + 3 * pl->nspec * csz;
        if (pl->mixed)
            k_phi_only<float2><<<blocks, KSPACE_THREADS, 0, pl->stream>>>(pl->nspec, (const float2*)pl->rho_hat,
                                                                           pl->G, (float2*)out);
        else
            k_phi_only<double2><<<blocks, KSPACE_THREADS, 0, pl->stream>>>(pl->nspec, (const double2*)pl->rho_hat,
                                                                            pl->G, (double2*)out);
        return hipGetLastError();
    }
    pl->epart_blocks = blocks;
    const int mode = (pl->p.diff == PPPM_DIFF_AD) ? 1 : 0;
    if (pl->mixed)
        k_solve<float2><<<blocks, KSPACE_THREADS, 0, pl->stream>>>(kg, pl->nspec, mode, (const float2*)pl->rho_hat,
                                                                    pl->G, (float2*)pl->spec, pl->epart);
    else
        k_solve<double2><<<blocks, KSPACE_THREADS, 0, pl->stream>>>(kg, pl->nspec, mode, (const double2*)pl->rho_hat,
                                                                     pl->G, (double2*)pl->spec, pl->epart);
    return hipGetLastError();
}

hipError_t launch_energy_final(pppm_plan_s* pl, double* energy_out)
{
    k_energy_final<<<1, 1024, 0, pl->stream>>>(energy_sums(pl, energy_out));
    return hipGetLastError();
}

hipError_t launch_copy_terms(pppm_plan_s* pl, double* out3)
{
    return hipMemcpyAsync(out3, pl->eterms + 1, 3 * sizeof(double), hipMemcpyDeviceToDevice, pl->stream);
}

}  // namespace pppm
