// C ABI of the MI355X PPPM library: parameter validation, plan lifetime,
// device scratch, rocFFT plans and the enqueue order of the steps
//   particle map -> make_rho -> Poisson (FFT, G multiply, energy, inverse
//   FFT) -> fieldforce,
// following the three-step PPPM evaluation of the paper (Section 2.1) with
// the per-atom stencil setup of Section 3.1 as its own step.
#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "device_common.h"
#include "params.h"
#include "pppm_internal.h"

#include <vector>

using namespace pppm;

namespace {

thread_local std::string g_last_error;

pppm_status fail(pppm_plan_s* pl, pppm_status st, const std::string& msg)
{
    if (pl)
        pl->last_error = msg;
    else
        g_last_error = msg;
    return st;
}

#define HIP_TRY(pl, call)                                                                      \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail((pl), PPPM_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define FFT_TRY(pl, call)                                                                          \
    do {                                                                                           \
        rocfft_status s_ = (call);                                                                 \
        if (s_ != rocfft_status_success)                                                           \
            return fail((pl), PPPM_ERR_FFT, std::string(#call) + ": rocfft status " + std::to_string((int)s_)); \
    } while (0)

constexpr size_t LDS_PREFERRED = 80 * 1024 - 1024;  // keeps two or more workgroups per CU
constexpr size_t LDS_STATIC = 1024;                 // static LDS of the kernels, rounded up

std::once_flag g_fft_once;
rocfft_status g_fft_setup = rocfft_status_success;


// The histogram form of the particle map needs the bins of all tiles in one
// block's LDS.
bool use_hist_map(const pppm_plan_s* pl, int64_t nbins)
{
    return nbins <= HIST_MAX_BINS && (size_t)nbins * sizeof(int) + LDS_STATIC <= pl->lds_limit;
}

// Sizes the bin arrays for nbins bins of `stride` entries each (grown when a
// finer tiling needs more, never shrunk); returns "" or the failure.  Fresh
// counters are zeroed on the plan's stream.
std::string ensure_bin_buffers(pppm_plan_s* pl, int64_t nbins, int stride)
{
    const int64_t nent = nbins * stride;
    if (nent > pl->bin_capacity) {
        const int64_t scan_blocks = (nent + SCAN_BLOCK - 1) / SCAN_BLOCK;
        int *c = nullptr, *o = nullptr, *sp = nullptr;
        if (hipMalloc((void**)&c, nent * sizeof(int)) != hipSuccess ||
            hipMalloc((void**)&o, (nent + 1) * sizeof(int)) != hipSuccess ||
            hipMalloc((void**)&sp, 2 * scan_blocks * sizeof(int)) != hipSuccess ||
            hipMemsetAsync(c, 0, nent * sizeof(int), pl->stream) != hipSuccess) {
            (void)hipGetLastError();
            for (int* b : {c, o, sp})
                if (b) (void)hipFree(b);
            return "out of device memory for the bin arrays";
        }
        for (int* b : {pl->count, pl->offsets, pl->scan_part})
            if (b) (void)hipFree(b);
        pl->count = c;
        pl->offsets = o;
        pl->scan_part = sp;
        pl->bin_capacity = nent;
    }
    const size_t hist_bytes = stride == 1 ? (size_t)HIST_MAX_BLOCKS * nbins * sizeof(int) : 0;
    if (hist_bytes > pl->hist_bytes) {
        int* h = nullptr;
        if (hipMalloc((void**)&h, hist_bytes) != hipSuccess) {
            (void)hipGetLastError();
            return "out of device memory for the bin histogram";
        }
        if (pl->hist) (void)hipFree(pl->hist);
        pl->hist = h;
        pl->hist_bytes = hist_bytes;
    }
    return "";
}

// Host evaluation of the stencil weights and their derivatives (the same
// centred polynomial pieces the kernels evaluate), for the weight table.
template <int PP>
void host_weights(double f, double* w, double* dw)
{
    using Cf = WeightPoly<PP>;
    const double g = f - 0.5, g2 = g * g;
    for (int j = 0; j < (PP + 1) / 2; ++j) {
        double e = 0.0, o = 0.0, de = 0.0, dq = 0.0;
        for (int m = PP - 1; m >= 0; --m) {
            if (m % 2 == 0) e = e * g2 + Cf::c[j][m];
            else o = o * g2 + Cf::c[j][m];
        }
        for (int m = PP - 2; m >= 0; --m) {
            if (m % 2 == 0) de = de * g2 + (m + 1) * Cf::c[j][m + 1];
            else dq = dq * g2 + (m + 1) * Cf::c[j][m + 1];
        }
        w[j] = e + g * o;
        dw[j] = de + g * dq;
        if (PP - 1 - j != j) {
            w[PP - 1 - j] = e - g * o;
            dw[PP - 1 - j] = g * dq - de;
        }
    }
}

void host_weights(int P, double f, double* w, double* dw)
{
    switch (P) {
    case 2: host_weights<2>(f, w, dw); break;
    case 3: host_weights<3>(f, w, dw); break;
    case 4: host_weights<4>(f, w, dw); break;
    case 5: host_weights<5>(f, w, dw); break;
    case 6: host_weights<6>(f, w, dw); break;
    default: host_weights<7>(f, w, dw); break;
    }
}

// make_rho's form for tile geometry g, in the mixed form.  The push form
// (k_spread_push + k_fold) issues about half the LDS atomics of the
// owner-computes form (no halo pulls, no clipped rows) and pays a second
// pass over the boxes.  Measured on the default tiles (make_rho, us, owner-
// computes against push): P = 7: 89 / 77 on 524,288 charges at 128^3;
// P = 6: 57.5 / 53 there, 499 / 412 on 4.2M charges at 256^3, 32 / 25.5 on
// 65,536 charges at 64^3; P = 5: 37.1 / 39.8 at 128^3 (512 tiles), 48.8 /
// 58.4 at 160^3 (1,000 tiles), but 21.4 / 18.5 at 64^3 with 64 tiles, where
// the owner-computes form's doubled atomics sit on a quarter of the CUs and
// the push form moves that work into a fold that spreads over all of them
// (and 331 / 293 at 256^3, 4,096 tiles); P = 4: 24.9 / 31.9 at 128^3.  So the
// push form at P >= 6, and at P = 5 when there are fewer tiles than CUs.
// PPPM_SPREAD=push takes the push form at any order, =visit never.  Only
// when the box fits the LDS; with alloc the box buffer is grown here, and if
// that fails the plan keeps to the owner-computes form.
void choose_spread_form(pppm_plan_s* pl, const MapGeo& g, bool alloc)
{
    pl->spread_push = false;
    if (!pl->mixed || pl->spread_mode == 1) return;
    if (pl->spread_mode == 0) {
        const int P = pl->p.order;
        if (P <= 4 || (P == 5 && g.ntiles >= pl->num_cu)) return;
    }
    if (spread_push_lds_bytes(g) > pl->lds_limit - LDS_STATIC) return;
    if (alloc) {
        const size_t bytes = (size_t)g.ntiles * spread_box_points(g) * sizeof(float);
        if (bytes > pl->box_bytes) {
            float* b = nullptr;
            if (hipMalloc((void**)&b, bytes) != hipSuccess) {
                (void)hipGetLastError();
                return;
            }
            if (pl->box) (void)hipFree(pl->box);
            pl->box = b;
            pl->box_bytes = bytes;
        }
    }
    pl->spread_push = true;
}

// Set the plan's tile shape (edges B[3]); returns "" or the reason it is not
// usable.  Updates the mesh geometry shared by all particle-side kernels.
// With alloc false (the allocation-free call) the bin arrays are left to
// the caller, which sizes them for the chosen geometry afterwards.
std::string set_tile(pppm_plan_s* pl, const int* B, size_t lds_budget, bool alloc = true)
{
    const int P = pl->p.order;
    MapGeo g = pl->geo;
    for (int d = 0; d < 3; ++d) {
        if (B[d] < 1 || B[d] > 64) return "tile edges must be in [1, 64]";
        if (!tile_edge_ok(g.K[d], B[d], P))
            return "tile edge " + std::to_string(B[d]) + " along axis " + std::to_string(d) +
                   " leaves a tile thinner than order - 1 points";
        g.B[d] = B[d] < g.K[d] ? B[d] : g.K[d];
        g.ntile[d] = (g.K[d] + g.B[d] - 1) / g.B[d];
    }
    g.ntiles = g.ntile[0] * g.ntile[1] * g.ntile[2];
    g.bin_stride = use_hist_map(pl, (int64_t)g.ntiles * NCLASS) ? 1 : NSUB;
    const size_t lds_s = spread_lds_bytes(g);
    const size_t lds_g = gather_lds_bytes(g, P, pl->ncomp, pl->rsize, 512);
    const size_t lds_a = gather_lds_bytes(g, P, 1, pl->rsize, 512);
    const size_t lim = pl->lds_limit - LDS_STATIC < lds_budget ? pl->lds_limit - LDS_STATIC : lds_budget;
    if ((int64_t)g.ntiles * NCLASS > pl->max_bins) return "tile too fine for the plan's bin arrays";
    if (lds_s > lim || lds_g > lim || lds_a > lim)
        return "tile needs " + std::to_string(lds_s > lds_g ? lds_s : lds_g) + " bytes of LDS";
    if (alloc) {
        const std::string why = ensure_bin_buffers(pl, (int64_t)g.ntiles * NCLASS, g.bin_stride);
        if (!why.empty()) return why;
        // The atomic form of the particle map counts into count[] and relies
        // on it starting at zero (its scan clears it again).  The histogram
        // form leaves its bin totals there, so a switch from that form
        // clears it.
        if (g.bin_stride == NSUB &&
            hipMemsetAsync(pl->count, 0, (size_t)g.ntiles * NCLASS * NSUB * sizeof(int), pl->stream) != hipSuccess) {
            (void)hipGetLastError();
            return "clearing the bin counters failed";
        }
    }
    choose_spread_form(pl, g, alloc);
    pl->geo = g;
    pl->nbins = (int64_t)g.ntiles * NCLASS;
    pl->stage = Stage::Empty;
    return "";
}

// Workgroup of the forward gather on the plan's tile: `want` threads or, when
// the tile's staged meshes and lane buffers would not fit the LDS with them,
// the most (a multiple of 64) that fit; a usable tile fits 512.
int fit_gather_threads(const pppm_plan_s* pl, int want)
{
    int t = want;
    while (t > 512 && gather_lds_bytes(pl->geo, pl->p.order, pl->ncomp, pl->rsize, t) + LDS_STATIC > pl->lds_limit)
        t -= 64;
    return t;
}

// Default forward-gather workgroup: 768 threads for the mixed ik gather (its
// three staged meshes leave one workgroup per CU; measured on 524,288
// charges at 128^3: 44.9 against 46.7 us at P = 5 and 94 against 112 us at
// P = 7 for 512 threads, 1024 threads 44.5 and 107 us), where the LDS allows;
// 512 for the others.
int default_gather_threads(const pppm_plan_s* pl)
{
    return (pl->mixed && pl->p.diff == PPPM_DIFF_IK) ? fit_gather_threads(pl, 768) : 512;
}

// Default tile: the first usable shape of a preference list, each axis split
// evenly.  Measured (mixed precision, whole step: particle map + make_rho +
// Poisson + fieldforce): ad keeps 32 x 16 x 8 (on the 524,288-charge 128^3
// system 32 x 8 x 16 was within noise of it at P = 5 and on the 4.2M-charge
// 256^3 system at P = 7 slower, 1.47 against 1.39 ms); ik takes 32 x 16 x 8
// with the full LDS (161 against 167 us at P = 5 on 128^3, 2.03 against
// 2.29 ms at P = 7 on 256^3, where the tiles that keep the gather's three
// staged meshes within 79 KiB of LDS were 32 x 8 x 8 and 16 x 8 x 8).
// Tiles stay at 4,096 points: 8,192-point tiles (32 x 16 x 16, 32 x 32 x 8)
// halve the bins and the spread's halo pulls but leave the gather one
// workgroup per CU, so they gain 2 % at P = 5 and 5 % at P = 7 on 128^3 and
// lose 4 % on the 4.2M-charge 256^3 system (64 x 16 x 8 gains there but
// doubles the mixed form's error, its coarse occupancy cells being wider
// along x).
std::string default_tile(pppm_plan_s* pl, bool alloc = true)
{
    static const int prefs_ad[][3] = {{32, 16, 8}, {32, 8, 8}, {16, 16, 8}, {16, 8, 8}, {8, 8, 8}, {8, 8, 4}, {4, 4, 4}};
    static const int prefs_ik[][3] = {{32, 16, 8}, {32, 8, 16}, {32, 8, 8}, {16, 16, 8},
                                      {16, 8, 8},  {8, 8, 8},   {8, 8, 4},  {4, 4, 4}};
    const bool ik = pl->p.diff == PPPM_DIFF_IK;
    const int (*prefs)[3] = ik ? prefs_ik : prefs_ad;
    const int nprefs = ik ? 8 : 7;
    std::string why;
    // first within the LDS size that keeps several workgroups per CU (the
    // mixed ik gather: anything the device holds, its best tiles need more),
    // then anything the device holds (small meshes that cannot be split)
    const size_t first = (ik && pl->mixed) ? pl->lds_limit : LDS_PREFERRED;
    for (size_t budget : {first, pl->lds_limit}) {
        for (int k = 0; k < nprefs; ++k) {
            const int* pref = prefs[k];
            int B[3];
            for (int d = 0; d < 3; ++d) B[d] = split_tile_edge(pl->geo.K[d], pref[d], pl->p.order);
            if (B[0] > 64 || B[1] > 64 || B[2] > 64) {
                why = "mesh axis too long for a single tile";
                continue;
            }
            why = set_tile(pl, B, budget, alloc);
            if (why.empty()) {
                pl->gather_cfg.threads = default_gather_threads(pl);
                return "";
            }
        }
    }
    return why;
}

template <typename T>
pppm_status dmalloc(pppm_plan_s* pl, T** ptr, size_t bytes)
{
    *ptr = nullptr;
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc((void**)ptr, bytes);
    if (e != hipSuccess) {
        *ptr = nullptr;
        (void)hipGetLastError();
        return fail(pl, PPPM_ERR_OOM, "hipMalloc(" + std::to_string(bytes) + "): " + hipGetErrorString(e));
    }
    return PPPM_OK;
}

// Builds the plan's weight table (PPPM_FLAG_WEIGHT_TABLE): T + 1 rows at
// f = i / T of the P weights and the P derivative weights, in the particle-
// side precision.
pppm_status build_weight_table(pppm_plan_s* pl)
{
    const uint32_t ts = (pl->p.flags >> 8) & 0xFFFFu;
    const int T = ts ? (int)ts : 5000;
    const int P = pl->p.order;
    std::vector<double> h((size_t)(T + 1) * 2 * P);
    for (int i = 0; i <= T; ++i) host_weights(P, (double)i / T, &h[(size_t)i * 2 * P], &h[(size_t)i * 2 * P + P]);
    std::vector<float> hf;
    const void* src = h.data();
    size_t bytes = h.size() * sizeof(double);
    if (pl->mixed) {
        hf.assign(h.begin(), h.end());
        src = hf.data();
        bytes = hf.size() * sizeof(float);
    }
    pppm_status st = dmalloc(pl, &pl->wtab, bytes);
    if (st != PPPM_OK) return st;
    const hipError_t e = hipMemcpy(pl->wtab, src, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(pl, PPPM_ERR_HIP, std::string("weight table upload: ") + hipGetErrorString(e));
    pl->geo.wtab = pl->wtab;
    pl->geo.wtab_n = T;
    return PPPM_OK;
}

void release(pppm_plan_s* pl)
{
    if (pl->fft_fwd) rocfft_plan_destroy(pl->fft_fwd);
    if (pl->fft_inv) rocfft_plan_destroy(pl->fft_inv);
    if (pl->fft_inv1) rocfft_plan_destroy(pl->fft_inv1);
    if (pl->fft_info) rocfft_execution_info_destroy(pl->fft_info);
    void* bufs[] = {pl->count, pl->offsets, pl->scan_part, pl->slot, pl->records, pl->perm, pl->qpart, pl->hist,
                    pl->rho, pl->rho_hat, pl->spec, pl->field, pl->G, pl->epart, pl->eterms, pl->flags, pl->wtab,
                    pl->sfc,   pl->fft_tw,  pl->fft_work, pl->box};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
}

pppm_status make_fft_plans(pppm_plan_s* pl)
{
    std::call_once(g_fft_once, [] { g_fft_setup = rocfft_setup(); });
    FFT_TRY(pl, g_fft_setup);
    const size_t lengths[3] = {(size_t)pl->geo.K[0], (size_t)pl->geo.K[1], (size_t)pl->geo.K[2]};
    // the mixed form transforms in FP32 both ways; the energy sum stays FP64
    const rocfft_precision inv_prec = pl->mixed ? rocfft_precision_single : rocfft_precision_double;
    FFT_TRY(pl, rocfft_plan_create(&pl->fft_fwd, rocfft_placement_notinplace, rocfft_transform_type_real_forward,
                                   inv_prec, 3, lengths, 1, nullptr));
    FFT_TRY(pl, rocfft_plan_create(&pl->fft_inv, rocfft_placement_notinplace, rocfft_transform_type_real_inverse,
                                   inv_prec, 3, lengths, (size_t)pl->ncomp, nullptr));
    if (pl->p.diff == PPPM_DIFF_IK)
        FFT_TRY(pl, rocfft_plan_create(&pl->fft_inv1, rocfft_placement_notinplace,
                                       rocfft_transform_type_real_inverse, inv_prec, 3, lengths, 1, nullptr));
    size_t w = 0, wi = 0;
    FFT_TRY(pl, rocfft_plan_get_work_buffer_size(pl->fft_fwd, &w));
    FFT_TRY(pl, rocfft_plan_get_work_buffer_size(pl->fft_inv, &wi));
    w = w > wi ? w : wi;
    if (pl->fft_inv1) {
        FFT_TRY(pl, rocfft_plan_get_work_buffer_size(pl->fft_inv1, &wi));
        w = w > wi ? w : wi;
    }
    FFT_TRY(pl, rocfft_execution_info_create(&pl->fft_info));
    FFT_TRY(pl, rocfft_execution_info_set_stream(pl->fft_info, pl->stream));
    if (w > 0) {
        pppm_status st = dmalloc(pl, &pl->fft_work, w);
        if (st != PPPM_OK) return st;
        pl->fft_work_bytes = w;
        FFT_TRY(pl, rocfft_execution_info_set_work_buffer(pl->fft_info, pl->fft_work, w));
    }
    return PPPM_OK;
}

// The part of plan creation that allocates nothing: parameters, device,
// mesh geometry, transform shapes and default launch sizes.
pppm_status init_plan_geometry(pppm_plan_s* pl, const pppm_params* params, void* hip_stream)
{
    pl->p = *params;
    pl->stream = (hipStream_t)hip_stream;
    pl->mixed = params->prec == PPPM_PREC_MIXED;
    pl->rsize = pl->mixed ? sizeof(float) : sizeof(double);
    pl->ncomp = params->diff == PPPM_DIFF_IK ? 3 : 1;
    hipError_t e = hipGetDevice(&pl->device);
    if (e != hipSuccess) return fail(pl, PPPM_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    int lds = 0;
    e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, pl->device);
    if (e != hipSuccess) return fail(pl, PPPM_ERR_HIP, std::string("hipDeviceGetAttribute: ") + hipGetErrorString(e));
    pl->lds_limit = (size_t)lds;
    int ncu = 0;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, pl->device);
    if (e != hipSuccess) return fail(pl, PPPM_ERR_HIP, std::string("hipDeviceGetAttribute: ") + hipGetErrorString(e));
    pl->num_cu = ncu > 0 ? ncu : 1;
    // PPPM_SPREAD=visit keeps make_rho to the owner-computes form, =push takes
    // the push form at every order whenever its box fits the LDS (for
    // comparisons); otherwise the form follows the order and the tile count
    const char* spread_env = std::getenv("PPPM_SPREAD");
    pl->spread_mode = !spread_env ? 0 : (std::strcmp(spread_env, "visit") == 0 ? 1 : (std::strcmp(spread_env, "push") == 0 ? 2 : 0));

    MapGeo& g = pl->geo;
    for (int d = 0; d < 3; ++d) {
        g.lo[d] = params->box_lo[d];
        g.K[d] = params->mesh[d];
        g.h[d] = params->box_len[d] / (double)params->mesh[d];
    }
    g.shift = 1.0 - 0.5 * params->order;
    g.halo = params->order - 1;
    g.check_finite = (params->flags & PPPM_FLAG_CHECK_FINITE) ? 1 : 0;
    pl->ncell = (int64_t)g.K[0] * g.K[1] * g.K[2];
    pl->nspec = (int64_t)(g.K[0] / 2 + 1) * g.K[1] * g.K[2];
    // finest tiling accepted: as many bins as tiles with edges of 4 points
    pl->max_bins = (int64_t)((g.K[0] + 3) / 4) * ((g.K[1] + 3) / 4) * ((g.K[2] + 3) / 4) * NCLASS;
    // power-of-two meshes whose transform blocks fit in LDS use the library's
    // own Poisson passes
    pl->own_fft = own_fft_supported(g.K, pl->mixed);
    if (pl->own_fft) {
        own_fft_shapes(pl);
        if (!own_fft_shapes_ok(pl) || own_fft_lds_max(pl) + LDS_STATIC > pl->lds_limit) pl->own_fft = false;
    }
    if (!pl->own_fft) pl->spec_len = pl->nspec;
    pl->spread_cfg.threads = 1024;
    pl->gather_cfg.threads = pl->adjoint_cfg.threads = 512;
    return PPPM_OK;
}

// Bytes of the plan's device buffers (other than the bin arrays, which
// follow the tiling).
struct BufferSizes {
    size_t records, qpart, rho, rho_hat, spec, field, G, epart, sfc, fft_tw;
};
BufferSizes buffer_sizes(const pppm_plan_s* pl)
{
    const MapGeo& g = pl->geo;
    const int64_t nmax = pl->p.max_particles;
    const size_t csz = pl->mixed ? sizeof(float2) : sizeof(double2);
    BufferSizes z{};
    z.records = nmax * (pl->mixed ? sizeof(float4) : sizeof(double4));
    z.qpart = 3 * ((nmax + MAP_THREADS - 1) / MAP_THREADS + 1) * sizeof(double);
    z.rho = pl->ncell * pl->rsize;
    z.rho_hat = pl->spec_len * csz;
    z.spec = (pl->ncomp + 1) * pl->spec_len * csz;
    z.field = (pl->ncomp + 1) * pl->ncell * pl->rsize;
    const int64_t g_len =
        pl->own_fft ? (int64_t)(g.K[0] / 2 + 1) * (g.K[1] / 2 + 1) * (g.K[2] / 2 + 1) : pl->nspec;
    z.G = g_len * sizeof(double);
    z.epart = ((pl->own_fft && pl->fz_blocks > 2048) ? pl->fz_blocks : 2048) * sizeof(double);
    z.sfc = (6 + 6 * (size_t)kspace_blocks(pl->nspec)) * sizeof(double);
    z.fft_tw = (size_t)(g.K[0] + g.K[1] + g.K[2]) * csz;
    return z;
}

// ---- scratch of the allocation-free call ---------------------------------
// One static array per GPU, holding every device buffer of the transient
// plan of pppm_compute_noalloc.  In host code its name stands for a host
// symbol: kernels and copies take the device address that
// hipGetSymbolAddress returns, looked up once per device.
__device__ __align__(256) unsigned char scratch[PPPM_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[MAX_DEVICES] = {};

unsigned char* device_scratch(int dev, std::string& why)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (dev < 0 || dev >= MAX_DEVICES) {
        why = "device index " + std::to_string(dev) + " out of range";
        return nullptr;
    }
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            why = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        g_scratch_ptr[dev] = (unsigned char*)ptr;
    }
    return g_scratch_ptr[dev];
}

// Zero n 32-bit words (a kernel rather than hipMemsetAsync, so that the call
// can be captured in a HIP graph).
__global__ void k_zero_words(unsigned* __restrict__ p, long long n)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Carves 256-byte aligned buffers out of the scratch array; `used` may run
// past the capacity, which the caller checks before any buffer is touched.
struct Carver {
    unsigned char* base;
    size_t used;
    template <typename T> void take(T** ptr, size_t bytes)
    {
        used = (used + 255) & ~(size_t)255;
        *ptr = (T*)(base + used);
        used += bytes > 0 ? bytes : 256;
    }
};

pppm_status check_plan(pppm_plan_s* pl)
{
    if (!pl) return fail(nullptr, PPPM_ERR_ARG, "plan is NULL");
    pl->last_error.clear();
    return PPPM_OK;
}

pppm_status do_particle_map(pppm_plan_s* pl, int64_t n, const void* pos, const void* q)
{
    if (n < 0 || n > pl->p.max_particles)
        return fail(pl, PPPM_ERR_ARG, "n = " + std::to_string(n) + " outside [0, max_particles = " +
                                          std::to_string(pl->p.max_particles) + "]");
    if (n > 0 && (!pos || !q)) return fail(pl, PPPM_ERR_ARG, "pos and q must not be NULL");
    pl->stage = Stage::Empty;
    pl->phi_valid = false;
    HIP_TRY(pl, launch_map_count(pl, n, pos, q));
    HIP_TRY(pl, launch_scan(pl));
    HIP_TRY(pl, launch_scatter(pl, n, pos, q));
    pl->n = n;
    pl->pos_ptr = pos;
    pl->q_ptr = q;
    pl->stage = Stage::Mapped;
    return PPPM_OK;
}

pppm_status do_make_rho(pppm_plan_s* pl, double* rho)
{
    if (pl->stage < Stage::Mapped) return fail(pl, PPPM_ERR_STATE, "make_rho before particle_map");
    HIP_TRY(pl, launch_spread(pl, rho));
    pl->stage = Stage::Spread;
    pl->phi_valid = false;
    return PPPM_OK;
}

pppm_status do_poisson(pppm_plan_s* pl, double* energy)
{
    if (pl->stage < Stage::Spread) return fail(pl, PPPM_ERR_STATE, "poisson before make_rho");
    if (pl->own_fft) {
        HIP_TRY(pl, launch_own_poisson(pl, false, energy));
    } else {
        void* in[1] = {pl->rho};
        void* out[1] = {pl->rho_hat};
        FFT_TRY(pl, rocfft_execute(pl->fft_fwd, in, out, pl->fft_info));
        HIP_TRY(pl, launch_kspace(pl, false));
        HIP_TRY(pl, launch_energy_final(pl, energy));
        void* sin_[1] = {pl->spec};
        void* fout[1] = {pl->field};
        FFT_TRY(pl, rocfft_execute(pl->fft_inv, sin_, fout, pl->fft_info));
    }
    HIP_TRY(pl, hipGetLastError());
    pl->stage = Stage::Solved;
    pl->phi_valid = (pl->p.diff == PPPM_DIFF_AD);
    return PPPM_OK;
}

pppm_status do_fieldforce(pppm_plan_s* pl, void* forces)
{
    if (pl->stage < Stage::Solved) return fail(pl, PPPM_ERR_STATE, "fieldforce before poisson");
    if (!forces) return fail(pl, PPPM_ERR_ARG, "forces is NULL");
    if (pl->n == 0) return PPPM_OK;
    HIP_TRY(pl, launch_gather(pl, pl->p.diff == PPPM_DIFF_IK ? GATHER_IK : GATHER_AD, forces, nullptr, nullptr));
    return PPPM_OK;
}

}  // namespace

extern "C" {

pppm_status pppm_validate(const pppm_params* params)
{
    std::string why;
    pppm_status st = validate_params(params, why);
    if (st != PPPM_OK) return fail(nullptr, st, why);
    return PPPM_OK;
}

pppm_status pppm_plan_create(const pppm_params* params, void* hip_stream, pppm_plan* out)
{
    if (!out) return fail(nullptr, PPPM_ERR_ARG, "out is NULL");
    *out = nullptr;
    std::string why;
    pppm_status st = validate_params(params, why);
    if (st != PPPM_OK) return fail(nullptr, st, why);

    auto* pl = new pppm_plan_s();
    auto bail = [&](pppm_status s) {
        g_last_error = pl->last_error;
        release(pl);
        delete pl;
        return s;
    };
    if ((st = init_plan_geometry(pl, params, hip_stream)) != PPPM_OK) return bail(st);
    const int64_t nmax = params->max_particles;
    const BufferSizes z = buffer_sizes(pl);
    hipError_t e;
    if ((st = dmalloc(pl, &pl->slot, nmax * sizeof(int))) != PPPM_OK ||
        (st = dmalloc(pl, &pl->records, z.records)) != PPPM_OK ||
        (st = dmalloc(pl, &pl->perm, nmax * sizeof(int))) != PPPM_OK ||
        (st = dmalloc(pl, &pl->qpart, z.qpart)) != PPPM_OK ||
        (st = dmalloc(pl, &pl->rho, z.rho)) != PPPM_OK ||
        (st = dmalloc(pl, &pl->rho_hat, z.rho_hat)) != PPPM_OK ||
        (st = dmalloc(pl, &pl->spec, z.spec)) != PPPM_OK ||
        (st = dmalloc(pl, &pl->field, z.field)) != PPPM_OK ||
        (st = dmalloc(pl, &pl->G, z.G)) != PPPM_OK ||
        (st = dmalloc(pl, &pl->epart, z.epart)) != PPPM_OK ||
        (st = dmalloc(pl, &pl->eterms, 10 * sizeof(double))) != PPPM_OK ||
        (st = dmalloc(pl, &pl->flags, sizeof(int))) != PPPM_OK)
        return bail(st);

    e = hipMemsetAsync(pl->flags, 0, sizeof(int), pl->stream);
    if (e == hipSuccess) e = hipMemsetAsync(pl->eterms, 0, 10 * sizeof(double), pl->stream);
    if (e != hipSuccess) {
        pl->last_error = std::string("hipMemsetAsync: ") + hipGetErrorString(e);
        return bail(PPPM_ERR_HIP);
    }
    e = launch_influence(pl);
    if (e != hipSuccess) {
        pl->last_error = std::string("influence function: ") + hipGetErrorString(e);
        return bail(PPPM_ERR_HIP);
    }
    if (params->flags & PPPM_FLAG_AD_SELF_FORCE) {
        if ((st = dmalloc(pl, &pl->sfc, z.sfc)) != PPPM_OK) return bail(st);
        e = launch_self_force_coef(pl);
        if (e != hipSuccess) {
            pl->last_error = std::string("self-force coefficients: ") + hipGetErrorString(e);
            return bail(PPPM_ERR_HIP);
        }
    }
    if (pl->own_fft) {
        if ((st = dmalloc(pl, &pl->fft_tw, z.fft_tw)) != PPPM_OK) return bail(st);
        e = launch_own_fft_twiddles(pl);
        if (e != hipSuccess) {
            pl->last_error = std::string("twiddle tables: ") + hipGetErrorString(e);
            return bail(PPPM_ERR_HIP);
        }
    } else if ((st = make_fft_plans(pl)) != PPPM_OK) {
        return bail(st);
    }
    if ((params->flags & PPPM_FLAG_WEIGHT_TABLE) && (st = build_weight_table(pl)) != PPPM_OK) return bail(st);

    {
        std::string bad = default_tile(pl);
        if (!bad.empty()) {
            pl->last_error = "no usable tile shape: " + bad;
            return bail(PPPM_ERR_MESH);
        }
    }
    e = hipStreamSynchronize(pl->stream);
    if (e != hipSuccess) {
        pl->last_error = std::string("plan setup: ") + hipGetErrorString(e);
        return bail(PPPM_ERR_HIP);
    }
    *out = pl;
    return PPPM_OK;
}

pppm_status pppm_plan_destroy(pppm_plan plan)
{
    if (!plan) return PPPM_OK;
    (void)hipStreamSynchronize(plan->stream);
    release(plan);
    delete plan;
    return PPPM_OK;
}

pppm_status pppm_particle_map(pppm_plan plan, int64_t n, const void* pos, const void* q)
{
    pppm_status st = check_plan(plan);
    if (st != PPPM_OK) return st;
    return do_particle_map(plan, n, pos, q);
}

pppm_status pppm_make_rho(pppm_plan plan, double* rho)
{
    pppm_status st = check_plan(plan);
    if (st != PPPM_OK) return st;
    return do_make_rho(plan, rho);
}

pppm_status pppm_poisson(pppm_plan plan, double* energy)
{
    pppm_status st = check_plan(plan);
    if (st != PPPM_OK) return st;
    return do_poisson(plan, energy);
}

pppm_status pppm_fieldforce(pppm_plan plan, void* forces)
{
    pppm_status st = check_plan(plan);
    if (st != PPPM_OK) return st;
    return do_fieldforce(plan, forces);
}

pppm_status pppm_compute(pppm_plan plan, int64_t n, const void* pos, const void* q, double* rho, double* energy,
                         void* forces)
{
    pppm_status st = check_plan(plan);
    if (st != PPPM_OK) return st;
    if ((st = do_particle_map(plan, n, pos, q)) != PPPM_OK) return st;
    if ((st = do_make_rho(plan, rho)) != PPPM_OK) return st;
    if ((st = do_poisson(plan, energy)) != PPPM_OK) return st;
    if (forces) return do_fieldforce(plan, forces);
    return PPPM_OK;
}

pppm_status pppm_energy_backward(pppm_plan plan, const double* grad_energy, int64_t n, const void* pos,
                                 const void* q, void* grad_pos, void* grad_q)
{
    pppm_status st = check_plan(plan);
    if (st != PPPM_OK) return st;
    pppm_plan_s* pl = plan;
    if (!grad_energy) return fail(pl, PPPM_ERR_ARG, "grad_energy is NULL");
    if (pl->stage < Stage::Solved || n != pl->n || pos != pl->pos_ptr || q != pl->q_ptr)
        return fail(pl, PPPM_ERR_STATE, "energy_backward needs a preceding compute on the same pos, q and n");
    if (n == 0 || (!grad_pos && !grad_q)) return PPPM_OK;
    // The binned records of the forward call are still those of (pos, q): the
    // adjoint gather reads them and recomputes the stencil weights, so the
    // gradient belongs to the same positions as the retained potential.
    if (!pl->phi_valid) {
        // ik plan: the potential mesh of the same influence function
        if (pl->own_fft) {
            HIP_TRY(pl, launch_own_poisson(pl, true, nullptr));
        } else {
            HIP_TRY(pl, launch_kspace(pl, true));
            const size_t csz = pl->mixed ? sizeof(float2) : sizeof(double2);
            void* sin_[1] = {(char*)pl->spec + 3 * pl->nspec * csz};
            void* fout[1] = {(char*)pl->field + 3 * pl->ncell * pl->rsize};
            FFT_TRY(pl, rocfft_execute(pl->fft_inv1, sin_, fout, pl->fft_info));
        }
        pl->phi_valid = true;
    }
    HIP_TRY(pl, launch_gather(pl, GATHER_ADJOINT, grad_pos, grad_q, grad_energy));
    return PPPM_OK;
}

pppm_status pppm_compute_noalloc(const pppm_params* params, void* hip_stream, int64_t n, const void* pos,
                                 const void* q, double* rho, double* energy, void* forces)
{
    std::string why;
    pppm_status st = validate_params(params, why);
    if (st != PPPM_OK) return fail(nullptr, st, why);
    if (params->flags & (PPPM_FLAG_WEIGHT_TABLE | PPPM_FLAG_CHECK_FINITE))
        return fail(nullptr, PPPM_ERR_ARG,
                    "the allocation-free call takes neither the weight table nor the checked mode (both need a plan)");
    if (n < 0 || n > params->max_particles)
        return fail(nullptr, PPPM_ERR_ARG, "n = " + std::to_string(n) + " outside [0, max_particles]");
    if (n > 0 && (!pos || !q)) return fail(nullptr, PPPM_ERR_ARG, "pos and q must not be NULL");

    // a transient plan on the host; every device buffer it uses lives in the
    // scratch array
    pppm_plan_s pl;
    if ((st = init_plan_geometry(&pl, params, hip_stream)) != PPPM_OK) return fail(nullptr, st, pl.last_error);
    if (!pl.own_fft)
        return fail(nullptr, PPPM_ERR_MESH,
                    "the allocation-free call needs a mesh of the library's own transforms (rocFFT plans allocate)");
    why = default_tile(&pl, false);
    if (!why.empty()) return fail(nullptr, PPPM_ERR_MESH, "no usable tile shape: " + why);
    unsigned char* base = device_scratch(pl.device, why);
    if (!base) return fail(nullptr, PPPM_ERR_HIP, why);

    const BufferSizes z = buffer_sizes(&pl);
    const int64_t nmax = params->max_particles;
    const int64_t nent = pl.nbins * pl.geo.bin_stride;
    Carver c{base, 0};
    c.take(&pl.count, nent * sizeof(int));
    c.take(&pl.offsets, (nent + 1) * sizeof(int));
    c.take(&pl.scan_part, 2 * ((nent + SCAN_BLOCK - 1) / SCAN_BLOCK) * sizeof(int));
    if (pl.geo.bin_stride == 1) {
        pl.hist_bytes = (size_t)HIST_MAX_BLOCKS * pl.nbins * sizeof(int);
        c.take(&pl.hist, pl.hist_bytes);
    }
    c.take(&pl.slot, nmax * sizeof(int));
    c.take(&pl.records, z.records);
    c.take(&pl.perm, nmax * sizeof(int));
    c.take(&pl.qpart, z.qpart);
    c.take(&pl.rho, z.rho);
    c.take(&pl.rho_hat, z.rho_hat);
    c.take(&pl.spec, z.spec);
    c.take(&pl.field, z.field);
    c.take(&pl.G, z.G);
    c.take(&pl.epart, z.epart);
    c.take(&pl.eterms, 10 * sizeof(double));
    c.take(&pl.flags, sizeof(int));
    c.take(&pl.fft_tw, z.fft_tw);
    if (params->flags & PPPM_FLAG_AD_SELF_FORCE) c.take(&pl.sfc, z.sfc);
    pl.bin_capacity = nent;
    if (pl.spread_push) {
        // the push form's boxes, when they fit beside the rest; otherwise
        // make_rho takes the owner-computes form
        const size_t before = c.used;
        c.take(&pl.box, (size_t)pl.geo.ntiles * spread_box_points(pl.geo) * sizeof(float));
        if (c.used > PPPM_NOALLOC_SCRATCH_BYTES) {
            c.used = before;
            pl.box = nullptr;
            pl.spread_push = false;
        }
    }
    if (c.used > PPPM_NOALLOC_SCRATCH_BYTES)
        return fail(nullptr, PPPM_ERR_ARG,
                    "these parameters need " + std::to_string(c.used) + " bytes of device scratch; the allocation-free "
                    "call holds " + std::to_string((size_t)PPPM_NOALLOC_SCRATCH_BYTES) +
                    " per GPU (use a plan, or fewer particles or mesh points)");

    // What must start at zero: the energy terms, the sticky flag and (for the
    // atomic form of the particle map) the bin counters.  The array keeps
    // the contents of the last call on this GPU.
    k_zero_words<<<1, 64, 0, pl.stream>>>((unsigned*)pl.eterms, 20);
    k_zero_words<<<1, 64, 0, pl.stream>>>((unsigned*)pl.flags, 1);
    if (pl.geo.bin_stride != 1)
        k_zero_words<<<(unsigned)std::min<int64_t>((nent + 255) / 256, 1024), 256, 0, pl.stream>>>(
            (unsigned*)pl.count, nent);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_influence(&pl);
    if (e == hipSuccess && (params->flags & PPPM_FLAG_AD_SELF_FORCE)) e = launch_self_force_coef(&pl);
    if (e == hipSuccess) e = launch_own_fft_twiddles(&pl);
    if (e != hipSuccess) return fail(nullptr, PPPM_ERR_HIP, std::string("plan kernels: ") + hipGetErrorString(e));
    if ((st = do_particle_map(&pl, n, pos, q)) != PPPM_OK || (st = do_make_rho(&pl, rho)) != PPPM_OK ||
        (st = do_poisson(&pl, energy)) != PPPM_OK || (forces && (st = do_fieldforce(&pl, forces)) != PPPM_OK))
        return fail(nullptr, st, pl.last_error);
    return PPPM_OK;
}

pppm_status pppm_energy_terms(pppm_plan plan, double* out3)
{
    pppm_status st = check_plan(plan);
    if (st != PPPM_OK) return st;
    if (!out3) return fail(plan, PPPM_ERR_ARG, "out3 is NULL");
    HIP_TRY(plan, launch_copy_terms(plan, out3));
    return PPPM_OK;
}

pppm_status pppm_sync(pppm_plan plan)
{
    pppm_status st = check_plan(plan);
    if (st != PPPM_OK) return st;
    HIP_TRY(plan, hipStreamSynchronize(plan->stream));
    int flag = 0;
    HIP_TRY(plan, hipMemcpy(&flag, plan->flags, sizeof(int), hipMemcpyDeviceToHost));
    if (flag) {
        HIP_TRY(plan, hipMemset(plan->flags, 0, sizeof(int)));
        return fail(plan, PPPM_ERR_NONFINITE, "a position or charge was not finite");
    }
    return PPPM_OK;
}

const char* pppm_status_string(pppm_status status)
{
    switch (status) {
    case PPPM_OK: return "PPPM_OK";
    case PPPM_ERR_ARG: return "PPPM_ERR_ARG: invalid argument";
    case PPPM_ERR_ORDER: return "PPPM_ERR_ORDER: order outside [2, 7]";
    case PPPM_ERR_MESH: return "PPPM_ERR_MESH: invalid mesh";
    case PPPM_ERR_DTYPE: return "PPPM_ERR_DTYPE: invalid precision or dtype";
    case PPPM_ERR_NONFINITE: return "PPPM_ERR_NONFINITE: non-finite input";
    case PPPM_ERR_OOM: return "PPPM_ERR_OOM: device allocation failed";
    case PPPM_ERR_HIP: return "PPPM_ERR_HIP: HIP runtime error";
    case PPPM_ERR_FFT: return "PPPM_ERR_FFT: rocFFT error";
    case PPPM_ERR_STATE: return "PPPM_ERR_STATE: call out of order";
    }
    return "unknown pppm_status";
}

const char* pppm_last_error(pppm_plan plan)
{
    return plan ? plan->last_error.c_str() : g_last_error.c_str();
}

pppm_status pppm_plan_set_launch(pppm_plan plan, int32_t which, const int32_t* tile, int32_t threads)
{
    pppm_status st = check_plan(plan);
    if (st != PPPM_OK) return st;
    if (which < 0 || which > 2 || !tile) return fail(plan, PPPM_ERR_ARG, "which must be 0, 1 or 2 and tile non-NULL");
    // the kernels' launch bounds
    const bool wide_gather = which == 1 && plan->mixed && plan->p.diff == PPPM_DIFF_IK;
    const int max_threads = (which == 0 || wide_gather) ? 1024 : 512;
    if (threads < 64 || threads > max_threads || threads % 64)
        return fail(plan, PPPM_ERR_ARG, "threads must be a multiple of 64 in [64, " + std::to_string(max_threads) +
                                            "] (1024 for make_rho and the mixed ik gather, 512 for the other gathers)");
    if (which == 1 && threads > 512) {
        // the wider gather's lane buffers on the requested tile, checked
        // before anything changes
        MapGeo tg = plan->geo;
        for (int d = 0; d < 3; ++d) tg.B[d] = tile[d] < tg.K[d] ? tile[d] : tg.K[d];
        if (gather_lds_bytes(tg, plan->p.order, plan->ncomp, plan->rsize, threads) + LDS_STATIC > plan->lds_limit)
            return fail(plan, PPPM_ERR_ARG,
                        "a gather of " + std::to_string(threads) + " threads needs more LDS than the device has");
    }
    const MapGeo keep = plan->geo;
    const int64_t keep_bins = plan->nbins;
    const Stage keep_stage = plan->stage;
    if (tile[0] != keep.B[0] || tile[1] != keep.B[1] || tile[2] != keep.B[2]) {
        const int B[3] = {tile[0], tile[1], tile[2]};
        std::string bad = set_tile(plan, B, plan->lds_limit);
        if (!bad.empty()) {
            plan->geo = keep;
            plan->nbins = keep_bins;
            plan->stage = keep_stage;
            return fail(plan, PPPM_ERR_ARG, bad);
        }
    }
    (which == 0 ? plan->spread_cfg : (which == 1 ? plan->gather_cfg : plan->adjoint_cfg)).threads = threads;
    // a new tile may not leave room for the forward gather's workgroup
    if (which != 1) plan->gather_cfg.threads = fit_gather_threads(plan, plan->gather_cfg.threads);
    return PPPM_OK;
}

pppm_status pppm_plan_get_launch(pppm_plan plan, int32_t which, int32_t* tile, int32_t* threads)
{
    pppm_status st = check_plan(plan);
    if (st != PPPM_OK) return st;
    if (which < 0 || which > 2 || !tile || !threads) return fail(plan, PPPM_ERR_ARG, "bad arguments");
    const LaunchCfg& c = which == 0 ? plan->spread_cfg : (which == 1 ? plan->gather_cfg : plan->adjoint_cfg);
    for (int d = 0; d < 3; ++d) tile[d] = plan->geo.B[d];
    *threads = c.threads;
    return PPPM_OK;
}

}  // extern "C"
