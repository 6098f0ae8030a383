// Fuzz driver for the library's host-side parameter logic (params.cpp),
// built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_sanitizers.py.  Exits non-zero on a broken invariant.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <random>
#include <string>

#include "params.h"

using pppm::split_tile_edge;
using pppm::tile_edge_ok;
using pppm::validate_params;

static int fail(const char* what, long a = 0, long b = 0, long c = 0)
{
    std::fprintf(stderr, "invariant broken: %s (%ld %ld %ld)\n", what, a, b, c);
    return 1;
}

int main()
{
    std::mt19937_64 rng(12345);
    const double specials[] = {0.0, -0.0, 1.0, -1.0, 1e-300, 1e300, std::numeric_limits<double>::infinity(),
                               -std::numeric_limits<double>::infinity(), std::numeric_limits<double>::quiet_NaN(),
                               std::numeric_limits<double>::denorm_min(), 170.0};
    const int ints[] = {0, 1, 2, 3, 7, 8, 64, 2048, 2049, -1, -2147483647 - 1, 2147483647};
    std::string why;
    int n_ok = 0;
    for (int it = 0; it < 200000; ++it) {
        pppm_params p{};
        auto dbl = [&]() { return (rng() & 3) ? std::ldexp((double)(rng() % 2001) - 1000.0, (int)(rng() % 20) - 10)
                                              : specials[rng() % (sizeof(specials) / sizeof(double))]; };
        auto in = [&]() { return (rng() & 1) ? (int)(rng() % 300) : ints[rng() % (sizeof(ints) / sizeof(int))]; };
        for (int d = 0; d < 3; ++d) {
            p.box_lo[d] = dbl();
            p.box_len[d] = dbl();
            p.mesh[d] = in();
        }
        p.order = (rng() & 1) ? 2 + (int)(rng() % 6) : in();
        p.g_ewald = dbl();
        p.coulomb_c = dbl();
        p.diff = (pppm_diff)((rng() & 3) ? rng() % 2 : in());
        p.prec = (pppm_prec)((rng() & 3) ? rng() % 2 : in());
        p.io_dtype = (pppm_dtype)((rng() & 3) ? rng() % 2 : in());
        p.max_particles = (rng() & 3) ? (int64_t)(rng() % 1000000) : (int64_t)rng();
        p.flags = (rng() & 1) ? (uint32_t)(rng() & 7) | ((uint32_t)(rng() % 70000) << 8) : (uint32_t)rng();
        why.clear();
        const pppm_status st = validate_params(&p, why);
        if (st == PPPM_OK) {
            ++n_ok;
            long cells = 1;
            for (int d = 0; d < 3; ++d) {
                if (!(std::isfinite(p.box_len[d]) && p.box_len[d] > 0 && std::isfinite(p.box_lo[d])))
                    return fail("accepted a bad box", d);
                if (p.mesh[d] < 2 || p.mesh[d] < p.order || p.mesh[d] > 2048) return fail("accepted a bad mesh", d);
                cells *= p.mesh[d];
            }
            if (cells > (1L << 30)) return fail("accepted too many mesh points", cells);
            if (p.order < 2 || p.order > 7) return fail("accepted a bad order", p.order);
            if (!(p.g_ewald > 0) || !std::isfinite(p.g_ewald) || !(p.coulomb_c != 0) || !std::isfinite(p.coulomb_c))
                return fail("accepted a bad split or constant");
            if (p.max_particles < 0 || p.max_particles > 2147483647LL) return fail("accepted a bad capacity");
        } else if (why.empty()) {
            return fail("error without a reason", st);
        }
    }
    for (int P = 2; P <= 7; ++P)
        for (int K = 2; K <= 2048; K += (K < 300 ? 1 : 37))
            for (int b = 1; b <= 64; ++b) {
                const int B = split_tile_edge(K, b, P);
                if (B < 1) return fail("edge below 1", K, b, P);
                if (B != K && (B > 64 || !tile_edge_ok(K, B, P))) return fail("unusable edge", K, b, P);
            }
    if (n_ok == 0) return fail("no parameter set accepted");
    std::printf("params fuzz ok: %d accepted\n", n_ok);
    return 0;
}
