/*
 * Plain FP64 CPU reference of the PPPM particle-mesh steps.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code with the GPU library.
 *
 * What it computes follows the paper's description of the three mapping
 * functions (Section 3.1): a loop over atoms, the stencil coefficients of each
 * atom as the product of three one-dimensional polynomials whose order equals
 * the stencil size, and a triple loop over the S^3 stencil points.  Map-Charge
 * adds q * coefficient into the grid; Distribute-Force ik multiplies three
 * field grids by the coefficient and sums them per atom; Distribute-Force ad
 * multiplies the scalar potential by three derivative coefficients.  The
 * one-dimensional polynomial is read as the cardinal B-spline of order P
 * (the Hockney-Eastwood charge assignment function the paper builds on,
 * Section 2.1).
 *
 * Everything is written as the definition: one particle at a time, one
 * stencil point at a time, no blocking and no reordering.  Mesh arrays are
 * C-ordered [Kz][Ky][Kx] (x fastest).
 */
#define _USE_MATH_DEFINES
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_ORDER 7

/*
 * Stencil placement for one coordinate (Section 3.1, reading of the paper:
 * grid point m sits at lo + m*h; the P stencil points of a charge at mesh
 * coordinate u start at s = floor(u + 1 - P/2), which centres odd orders on
 * the nearest grid point and straddles the charge for even orders).
 * Returns the unwrapped start s and the fraction f = t - s in [0, 1).
 */
static void map_axis(double x, double lo, double len, int K, int P,
                     long *s_out, double *f_out)
{
    double h = len / (double)K;
    double u = (x - lo) / h;                 /* mesh coordinate */
    u = u - (double)K * floor(u / (double)K); /* periodic wrap into [0, K) */
    if (u < 0.0) u += (double)K;
    if (u >= (double)K) u -= (double)K;
    double t = u + 1.0 - 0.5 * (double)P;
    double s = floor(t);
    *s_out = (long)s;
    *f_out = t - s;
}

static long wrap_index(long i, int K)
{
    long r = i % K;
    return r < 0 ? r + K : r;
}

/*
 * Cardinal B-spline values a[k] = M_n(f + k), k = 0..n-1, from the two-term
 * recursion M_1 = 1 on [0,1),
 *   M_n(x) = [x M_{n-1}(x) + (n - x) M_{n-1}(x - 1)] / (n - 1).
 */
static void bspline_values(int n, double f, double *a)
{
    double prev[ORACLE_MAX_ORDER + 1];
    a[0] = 1.0;
    for (int m = 2; m <= n; ++m) {
        for (int k = 0; k < m - 1; ++k) prev[k] = a[k];
        for (int k = 0; k < m; ++k) {
            double left = (k < m - 1) ? prev[k] : 0.0;   /* M_{m-1}(f + k)     */
            double right = (k >= 1) ? prev[k - 1] : 0.0; /* M_{m-1}(f + k - 1) */
            a[k] = ((f + k) * left + ((double)m - f - k) * right) / (double)(m - 1);
        }
    }
}

/*
 * Stencil coefficients of one axis: w[j] is the weight of mesh point s + j,
 * w[j] = M_P(f + P - 1 - j); dw[j] = d w[j] / du, from
 * M_P'(x) = M_{P-1}(x) - M_{P-1}(x - 1).
 */
void oracle_weights(int P, double f, double *w, double *dw)
{
    double aP[ORACLE_MAX_ORDER + 1], aQ[ORACLE_MAX_ORDER + 1];
    bspline_values(P, f, aP);
    for (int j = 0; j < P; ++j) w[j] = aP[P - 1 - j];
    if (!dw) return;
    bspline_values(P - 1, f, aQ);
    for (int j = 0; j < P; ++j) {
        int k1 = P - 1 - j, k2 = P - 2 - j;
        double a = (k1 <= P - 2) ? aQ[k1] : 0.0;
        double b = (k2 >= 0) ? aQ[k2] : 0.0;
        dw[j] = a - b;
    }
}

/*
 * Weights of one particle's stencil.  table = 0: at its fraction f.  table =
 * T > 0: the tabulated variant of the mapping functions (Section 3.1), the
 * weights read from a table of their values at f = i / T, i = 0..T, nearest
 * entry; that is the weights at f rounded to the nearest multiple of 1 / T.
 */
static void stencil_at(int P, double f, int table, double *w, double *dw)
{
    if (table > 0) f = floor(f * (double)table + 0.5) / (double)table;
    oracle_weights(P, f, w, dw);
}

/* Per-particle stencil start (unwrapped) and fraction for all three axes. */
void oracle_particle_map(int64_t n, const double *pos, const double *lo,
                         const double *len, const int32_t *K, int P,
                         int64_t *s, double *f)
{
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            long sd;
            map_axis(pos[3 * i + d], lo[d], len[d], K[d], P, &sd, &f[3 * i + d]);
            s[3 * i + d] = sd;
        }
}

/* Map-Charge: rho_m = sum_i q_i wx wy wz over each particle's P^3 stencil. */
void oracle_make_rho(int64_t n, const double *pos, const double *q,
                     const double *lo, const double *len, const int32_t *K,
                     int P, int table, double *rho)
{
    const long Kx = K[0], Ky = K[1], Kz = K[2];
    memset(rho, 0, sizeof(double) * (size_t)(Kx * Ky * Kz));
    for (int64_t i = 0; i < n; ++i) {
        long s[3];
        double f[3], w[3][ORACLE_MAX_ORDER];
        for (int d = 0; d < 3; ++d) {
            map_axis(pos[3 * i + d], lo[d], len[d], K[d], P, &s[d], &f[d]);
            stencil_at(P, f[d], table, w[d], NULL);
        }
        for (int jz = 0; jz < P; ++jz)
            for (int jy = 0; jy < P; ++jy)
                for (int jx = 0; jx < P; ++jx) {
                    long mx = wrap_index(s[0] + jx, (int)Kx);
                    long my = wrap_index(s[1] + jy, (int)Ky);
                    long mz = wrap_index(s[2] + jz, (int)Kz);
                    rho[(mz * Ky + my) * Kx + mx] += q[i] * w[0][jx] * w[1][jy] * w[2][jz];
                }
    }
}

/*
 * Distribute-Force ik: F_i = q_i * sum over the stencil of wx wy wz E_m,
 * with E = (Ex, Ey, Ez) the three field meshes.
 */
void oracle_fieldforce_ik(int64_t n, const double *pos, const double *q,
                          const double *lo, const double *len, const int32_t *K,
                          int P, int table, const double *ex, const double *ey,
                          const double *ez, double *force)
{
    const long Kx = K[0], Ky = K[1];
    for (int64_t i = 0; i < n; ++i) {
        long s[3];
        double f[3], w[3][ORACLE_MAX_ORDER];
        for (int d = 0; d < 3; ++d) {
            map_axis(pos[3 * i + d], lo[d], len[d], K[d], P, &s[d], &f[d]);
            stencil_at(P, f[d], table, w[d], NULL);
        }
        double acc[3] = {0.0, 0.0, 0.0};
        for (int jz = 0; jz < P; ++jz)
            for (int jy = 0; jy < P; ++jy)
                for (int jx = 0; jx < P; ++jx) {
                    long mx = wrap_index(s[0] + jx, K[0]);
                    long my = wrap_index(s[1] + jy, K[1]);
                    long mz = wrap_index(s[2] + jz, K[2]);
                    long m = (mz * Ky + my) * Kx + mx;
                    double c = w[0][jx] * w[1][jy] * w[2][jz];
                    acc[0] += c * ex[m];
                    acc[1] += c * ey[m];
                    acc[2] += c * ez[m];
                }
        for (int d = 0; d < 3; ++d) force[3 * i + d] = q[i] * acc[d];
    }
}

/*
 * Distribute-Force ad: the gradient of the interpolated potential.  For axis
 * d the coefficient is the stencil product with the d-axis factor replaced
 * by its derivative dw/du; dividing by h_d turns d/du into d/dx_d.
 *   F_i = -q_i * (sum dwx wy wz phi / hx, sum wx dwy wz phi / hy,
 *                 sum wx wy dwz phi / hz).
 * Also returns pot_i = sum wx wy wz phi, the potential at the particle.
 */
void oracle_fieldforce_ad(int64_t n, const double *pos, const double *q,
                          const double *lo, const double *len, const int32_t *K,
                          int P, int table, const double *phi, double *force, double *pot)
{
    const long Kx = K[0], Ky = K[1];
    for (int64_t i = 0; i < n; ++i) {
        long s[3];
        double f[3], w[3][ORACLE_MAX_ORDER], dw[3][ORACLE_MAX_ORDER];
        for (int d = 0; d < 3; ++d) {
            map_axis(pos[3 * i + d], lo[d], len[d], K[d], P, &s[d], &f[d]);
            stencil_at(P, f[d], table, w[d], dw[d]);
        }
        double gx = 0.0, gy = 0.0, gz = 0.0, p = 0.0;
        for (int jz = 0; jz < P; ++jz)
            for (int jy = 0; jy < P; ++jy)
                for (int jx = 0; jx < P; ++jx) {
                    long mx = wrap_index(s[0] + jx, K[0]);
                    long my = wrap_index(s[1] + jy, K[1]);
                    long mz = wrap_index(s[2] + jz, K[2]);
                    double v = phi[(mz * Ky + my) * Kx + mx];
                    gx += dw[0][jx] * w[1][jy] * w[2][jz] * v;
                    gy += w[0][jx] * dw[1][jy] * w[2][jz] * v;
                    gz += w[0][jx] * w[1][jy] * dw[2][jz] * v;
                    p += w[0][jx] * w[1][jy] * w[2][jz] * v;
                }
        double hx = len[0] / K[0], hy = len[1] / K[1], hz = len[2] / K[2];
        force[3 * i + 0] = -q[i] * gx / hx;
        force[3 * i + 1] = -q[i] * gy / hy;
        force[3 * i + 2] = -q[i] * gz / hz;
        if (pot) pot[i] = p;
    }
}

/*
 * Influence function of the Poisson step on the full mesh, C order
 * [Kz][Ky][Kx], FFT index order.  The paper leaves the Green function
 * unspecified; reading: the optimal influence function for the order-P
 * B-spline assignment (minimum RMS force error), with
 *   U(k) = prod_d sinc(k_d h_d / 2)^P,  R(k) = 4 pi exp(-k^2/4g^2) / k^2,
 *   k_m = k + 2 pi m / h over aliases |m_d| <= alias,
 *   ik: G = sum_m U^2(k_m) (k . k_m) R(k_m) / (|k|^2 [sum_m U^2(k_m)]^2)
 *   ad: G = sum_m U^2(k_m) |k_m|^2 R(k_m) / ([sum_m U^2(k_m)] [sum_m |k_m|^2 U^2(k_m)])
 * and G(0) = 0.  diff: 0 = ik, 1 = ad.
 */
static double sinc(double x) { return x == 0.0 ? 1.0 : sin(x) / x; }

static double wavenumber(long k, long K, double len)
{
    long n = (2 * k < K) ? k : k - K; /* FFT order: n in [-K/2, K/2) */
    return 2.0 * M_PI * (double)n / len;
}

void oracle_influence_function(const double *len, const int32_t *K, int P,
                               double g, int diff, int alias, double *G)
{
    const long Kd[3] = {K[0], K[1], K[2]};
    const int na = 2 * alias + 1;
    /* Per axis, index and alias: the aliased wavenumber q, the assignment
     * factor sinc(q h / 2)^(2P) and the screening factor exp(-q^2 / 4g^2).
     * U^2 and exp(-|q|^2 / 4g^2) are products of these per-axis factors. */
    double *qa[3], *ua[3], *ea[3];
    for (int d = 0; d < 3; ++d) {
        const double h = len[d] / Kd[d];
        qa[d] = malloc(sizeof(double) * Kd[d] * na);
        ua[d] = malloc(sizeof(double) * Kd[d] * na);
        ea[d] = malloc(sizeof(double) * Kd[d] * na);
        for (long i = 0; i < Kd[d]; ++i)
            for (int m = 0; m < na; ++m) {
                double q = wavenumber(i, Kd[d], len[d]) + 2.0 * M_PI * (m - alias) / h;
                qa[d][i * na + m] = q;
                ua[d][i * na + m] = pow(sinc(0.5 * q * h), 2 * P);
                ea[d][i * na + m] = exp(-q * q / (4.0 * g * g));
            }
    }
    #pragma omp parallel for schedule(dynamic)
    for (long iz = 0; iz < Kd[2]; ++iz)
        for (long iy = 0; iy < Kd[1]; ++iy)
            for (long ix = 0; ix < Kd[0]; ++ix) {
                double kx = wavenumber(ix, Kd[0], len[0]);
                double ky = wavenumber(iy, Kd[1], len[1]);
                double kz = wavenumber(iz, Kd[2], len[2]);
                double k2 = kx * kx + ky * ky + kz * kz;
                double num = 0.0, sum_u2 = 0.0, sum_k2u2 = 0.0;
                for (int mz = 0; mz < na; ++mz)
                    for (int my = 0; my < na; ++my)
                        for (int mx = 0; mx < na; ++mx) {
                            double qx = qa[0][ix * na + mx], qy = qa[1][iy * na + my], qz = qa[2][iz * na + mz];
                            double u2 = ua[0][ix * na + mx] * ua[1][iy * na + my] * ua[2][iz * na + mz];
                            double q2 = qx * qx + qy * qy + qz * qz;
                            double ref = q2 > 0.0 ? 4.0 * M_PI * ea[0][ix * na + mx] * ea[1][iy * na + my] *
                                                    ea[2][iz * na + mz] / q2
                                                  : 0.0;
                            sum_u2 += u2;
                            sum_k2u2 += q2 * u2;
                            if (diff == 0)
                                num += u2 * (kx * qx + ky * qy + kz * qz) * ref;
                            else
                                num += u2 * q2 * ref;
                        }
                double v = 0.0;
                if (k2 > 0.0)
                    v = (diff == 0) ? num / (k2 * sum_u2 * sum_u2) : num / (sum_u2 * sum_k2u2);
                G[(iz * Kd[1] + iy) * Kd[0] + ix] = v;
            }
    for (int d = 0; d < 3; ++d) {
        free(qa[d]);
        free(ua[d]);
        free(ea[d]);
    }
}
