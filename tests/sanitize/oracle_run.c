/* Driver for the C oracle (oracle/oracle.c) on small systems, built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitizers.py:
 * every order, meshes down to the order, positions on the faces and far
 * outside the box.  Exits non-zero if the mesh charge does not sum to the
 * total charge. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_weights(int P, double f, double *w, double *dw);
void oracle_particle_map(int64_t n, const double *pos, const double *lo, const double *len, const int32_t *K,
                         int P, int64_t *s, double *f);
void oracle_make_rho(int64_t n, const double *pos, const double *q, const double *lo, const double *len,
                     const int32_t *K, int P, int table, double *rho);
void oracle_fieldforce_ik(int64_t n, const double *pos, const double *q, const double *lo, const double *len,
                          const int32_t *K, int P, int table, const double *ex, const double *ey, const double *ez,
                          double *force);
void oracle_fieldforce_ad(int64_t n, const double *pos, const double *q, const double *lo, const double *len,
                          const int32_t *K, int P, int table, const double *phi, double *force, double *pot);
void oracle_influence_function(const double *len, const int32_t *K, int P, double g, int diff, int alias,
                               double *G);

static double urand(unsigned *s)
{
    *s = *s * 1664525u + 1013904223u;
    return (double)(*s >> 8) / 16777216.0;
}

int main(void)
{
    unsigned seed = 7;
    const double lo[3] = {-3.0, 2.0, 0.5}, len[3] = {11.0, 13.0, 7.5};
    enum { N = 64 };
    double pos[3 * N], q[N], force[3 * N], pot[N], w[8], dw[8];
    int64_t s[3 * N];
    double f[3 * N];
    for (int P = 2; P <= 7; ++P) {
        const int32_t meshes[3][3] = {{P, P + 1, 9}, {8, 8, 8}, {13, 7 > P ? 7 : P, 11}};
        for (int mi = 0; mi < 3; ++mi) {
            const int32_t *K = meshes[mi];
            const long nc = (long)K[0] * K[1] * K[2];
            double *rho = malloc(sizeof(double) * nc), *ex = malloc(sizeof(double) * nc);
            double *ey = malloc(sizeof(double) * nc), *ez = malloc(sizeof(double) * nc);
            double *G = malloc(sizeof(double) * nc);
            double qsum = 0.0;
            for (int i = 0; i < N; ++i) {
                for (int d = 0; d < 3; ++d) pos[3 * i + d] = lo[d] + len[d] * (urand(&seed) * 5.0 - 2.0);
                q[i] = urand(&seed) - 0.5;
                qsum += q[i];
            }
            for (int d = 0; d < 3; ++d) {
                pos[d] = lo[d];
                pos[3 + d] = lo[d] + len[d];
                pos[6 + d] = lo[d] - 1e-300;
            }
            for (long m = 0; m < nc; ++m) {
                ex[m] = urand(&seed);
                ey[m] = urand(&seed);
                ez[m] = urand(&seed);
            }
            oracle_particle_map(N, pos, lo, len, K, P, s, f);
            oracle_make_rho(N, pos, q, lo, len, K, P, 0, rho);
            oracle_make_rho(N, pos, q, lo, len, K, P, 500, rho);
            double rsum = 0.0;
            for (long m = 0; m < nc; ++m) rsum += rho[m];
            if (fabs(rsum - qsum) > 1e-12) {
                fprintf(stderr, "mesh charge %g != total charge %g (P=%d)\n", rsum, qsum, P);
                return 1;
            }
            oracle_fieldforce_ik(N, pos, q, lo, len, K, P, 0, ex, ey, ez, force);
            oracle_fieldforce_ad(N, pos, q, lo, len, K, P, 0, ex, force, pot);
            oracle_fieldforce_ad(N, pos, q, lo, len, K, P, 5000, ex, force, NULL);
            oracle_influence_function(len, K, P, 0.45, 0, 2, G);
            oracle_influence_function(len, K, P, 0.45, 1, 2, G);
            for (int k = 0; k <= 20; ++k) oracle_weights(P, k / 20.0, w, dw);
            free(rho);
            free(ex);
            free(ey);
            free(ez);
            free(G);
        }
    }
    printf("oracle run ok\n");
    return 0;
}
