// Host-only parameter logic of the MI355X PPPM library: validation of a
// parameter set and the tile-edge rules of the launch geometry.  Plain C++
// (no HIP), so that it also builds with the host compiler alone.
#include "params.h"

#include <cmath>
#include <cstdint>
#include <cstring>

namespace pppm {

namespace {
constexpr int64_t MAX_CELLS = int64_t(1) << 30;
constexpr int MAX_MESH = 2048;

// The integer a C caller stored in an enum field.  C allows any int there,
// but in C++ loading an enum object that holds a value outside the range of
// its enumerators is undefined, so the check reads the bytes instead.
template <typename E>
int32_t raw_enum(const E& field)
{
    static_assert(sizeof(E) == sizeof(int32_t), "C enums are int-sized here");
    int32_t v;
    std::memcpy(&v, &field, sizeof v);
    return v;
}
}  // namespace

pppm_status validate_params(const pppm_params* p, std::string& why)
{
    if (!p) {
        why = "params is NULL";
        return PPPM_ERR_ARG;
    }
    if (p->order < 2 || p->order > 7) {
        why = "order must be in [2, 7], got " + std::to_string(p->order);
        return PPPM_ERR_ORDER;
    }
    int64_t cells = 1;
    for (int d = 0; d < 3; ++d) {
        if (!(std::isfinite(p->box_len[d]) && p->box_len[d] > 0.0) || !std::isfinite(p->box_lo[d])) {
            why = "box_lo must be finite and box_len positive and finite";
            return PPPM_ERR_ARG;
        }
        const int K = p->mesh[d];
        if (K < 2 || K < p->order || K > MAX_MESH) {
            why = "mesh[" + std::to_string(d) + "] = " + std::to_string(K) + " must be in [max(2, order), 2048]";
            return PPPM_ERR_MESH;
        }
        cells *= K;
    }
    if (cells > MAX_CELLS) {
        why = "more than 2^30 mesh points";
        return PPPM_ERR_MESH;
    }
    if (!(std::isfinite(p->g_ewald) && p->g_ewald > 0.0)) {
        why = "g_ewald must be positive and finite";
        return PPPM_ERR_ARG;
    }
    if (!std::isfinite(p->coulomb_c) || p->coulomb_c == 0.0) {
        why = "coulomb_c must be finite and non-zero";
        return PPPM_ERR_ARG;
    }
    if (raw_enum(p->diff) != PPPM_DIFF_IK && raw_enum(p->diff) != PPPM_DIFF_AD) {
        why = "diff must be PPPM_DIFF_IK or PPPM_DIFF_AD";
        return PPPM_ERR_ARG;
    }
    if (raw_enum(p->prec) != PPPM_PREC_FP64 && raw_enum(p->prec) != PPPM_PREC_MIXED) {
        why = "prec must be PPPM_PREC_FP64 or PPPM_PREC_MIXED";
        return PPPM_ERR_DTYPE;
    }
    if (raw_enum(p->io_dtype) != PPPM_F32 && raw_enum(p->io_dtype) != PPPM_F64) {
        why = "io_dtype must be PPPM_F32 or PPPM_F64";
        return PPPM_ERR_DTYPE;
    }
    if (p->max_particles < 0 || p->max_particles > 2147483647LL) {
        why = "max_particles must be in [0, 2^31 - 1]";
        return PPPM_ERR_ARG;
    }
    if (p->flags & ~(PPPM_FLAG_CHECK_FINITE | PPPM_FLAG_WEIGHT_TABLE | PPPM_FLAG_AD_SELF_FORCE |
                     PPPM_WEIGHT_TABLE_SIZE(0xFFFF))) {
        why = "unknown flag bits";
        return PPPM_ERR_ARG;
    }
    if ((p->flags & PPPM_FLAG_AD_SELF_FORCE) && raw_enum(p->diff) != PPPM_DIFF_AD) {
        why = "PPPM_FLAG_AD_SELF_FORCE needs diff = PPPM_DIFF_AD";
        return PPPM_ERR_ARG;
    }
    const uint32_t tsize = (p->flags >> 8) & 0xFFFFu;
    if (tsize != 0 && !(p->flags & PPPM_FLAG_WEIGHT_TABLE)) {
        why = "a weight-table size needs PPPM_FLAG_WEIGHT_TABLE";
        return PPPM_ERR_ARG;
    }
    if (tsize != 0 && tsize < 16) {
        why = "weight-table size must be at least 16";
        return PPPM_ERR_ARG;
    }
    return PPPM_OK;
}

// A tile edge B along an axis of K points is usable when the axis is a single
// tile (B >= K), or when every tile, the last (possibly thinner) one
// included, is at least P - 1 points thick, so that a stencil only ever
// reaches into the next tile.
bool tile_edge_ok(int K, int B, int P)
{
    if (B >= K) return true;
    const int rem = K % B;
    return B >= P - 1 && (rem == 0 || rem >= P - 1);
}

// Edge for an axis of K points near a preferred edge b: b itself when the
// last tile keeps at least P - 1 points (edges that are multiples of 4 keep
// the gather's 16-byte staging loads), else about K / b equal tiles, fewer if
// the last one would be thinner than P - 1.
int split_tile_edge(int K, int b, int P)
{
    // the preferred edge itself when it fits (a thinner last tile is fine)
    if (b < K && tile_edge_ok(K, b, P)) return b;
    int n = (K + b / 2) / b;
    if (n < 1) n = 1;
    for (; n > 1; --n) {
        const int B = (K + n - 1) / n;
        if (B <= 64 && tile_edge_ok(K, B, P)) return B;
    }
    return K;  // a single tile
}

}  // namespace pppm
