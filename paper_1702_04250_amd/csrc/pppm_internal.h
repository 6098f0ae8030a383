// Internal declarations of the MI355X PPPM library: plan state, launch
// geometry and the host launchers of the HIP kernels.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <cstdint>
#include <string>

#include "energy_sum.h"
#include "pppm.h"

namespace pppm {

// Charges are binned by the workgroup tile (a box of at most B_x x B_y x B_z
// mesh points) that holds their stencil start, and within a tile by a halo class:
// bit d is set when the stencil start lies within P - 1 points of the tile's
// upper face along d, i.e. when the stencil reaches into the next tile along
// d.  Each tile thus owns 8 consecutive bins.
constexpr int NCLASS = 8;
// Each bin is counted in NSUB sub-bins (picked by the particle index), so
// that the device-scope atomic counters of the particle map see NSUB times
// less contention.  The sub-bins of a bin are adjacent in the binned order:
// bin b starts at offsets[b * NSUB].
constexpr int NSUB = 16;
// Histogram form of the particle map (used when a tile's bins fit in LDS):
// HIST_THREADS-thread blocks each bin a chunk of consecutive charges in an
// LDS histogram and rank them there, so no device-scope atomics are needed.
constexpr int HIST_THREADS = 1024;
constexpr int HIST_MAX_BINS = 32768;   // LDS ints of one block
constexpr int HIST_MAX_BLOCKS = 256;
constexpr int HIST_CHUNK = 2048;       // target charges per block
constexpr int MAP_THREADS = 256;
constexpr int SCAN_THREADS = 1024;
constexpr int SCAN_ITEMS = 4;  // counts per thread per scan block
constexpr int SCAN_BLOCK = SCAN_THREADS * SCAN_ITEMS;
constexpr int KSPACE_THREADS = 256;

// Geometry shared by the particle-side kernels (passed by value).
struct MapGeo {
    double lo[3];
    double h[3];      // L / K, the same double the host computes
    double shift;     // 1 - P/2: stencil start s = floor(u + shift)
    int K[3];
    int B[3];         // tile edge in mesh points; the last tile of an axis may be thinner
    int ntile[3];     // tiles per axis, ceil(K / B)
    int ntiles;
    int halo;         // P - 1
    int check_finite;
    int bin_stride;   // offsets entries per bin: 1 (histogram map) or NSUB (atomic map)
    const void* wtab; // stencil-weight table of type R ([wtab_n + 1][2P]) or null: polynomials
    int wtab_n;       // table intervals T
};

struct LaunchCfg {
    int threads;
};

enum class Stage { Empty = 0, Mapped = 1, Spread = 2, Solved = 3 };

}  // namespace pppm

struct pppm_plan_s {
    pppm_params p{};
    hipStream_t stream = nullptr;
    int device = 0;
    size_t lds_limit = 65536;
    int num_cu = 256;          // compute units of the plan's device

    pppm::MapGeo geo{};
    int64_t ncell = 0;   // Kx Ky Kz
    int64_t nspec = 0;   // Kz Ky (Kx/2 + 1): half spectrum of a real transform
    int64_t nbins = 0;   // tiles x NCLASS
    int64_t max_bins = 0;      // most bins a tiling may have (tiles of edge 4)
    int64_t bin_capacity = 0;  // entries the count / offset arrays hold
    size_t hist_bytes = 0;     // bytes of the per-block histogram buffer
    int ncomp = 1;       // field meshes of the forward gather: 3 (ik) or 1 (ad)
    bool mixed = true;
    size_t rsize = 4;    // bytes of the particle-side real type (float / double)

    // device buffers owned by the plan
    int* count = nullptr;      // [nbins * bin_stride] charges per (sub-)bin (kept zero between calls)
    int* offsets = nullptr;    // [nbins * bin_stride + 1] exclusive prefix of count
    int* scan_part = nullptr;  // [2 * ceil(nbins * bin_stride / SCAN_BLOCK)] chunk sums, then chunk maxima
    int* slot = nullptr;       // [max_particles] rank of a particle within its sub-bin
    void* records = nullptr;   // [max_particles] float4 / double4 (t_x, t_y, t_z, q) in binned order;
                               // t = stencil start within the tile + fraction
    int* perm = nullptr;       // [max_particles] binned position -> caller index
    double* qpart = nullptr;   // [3 * map blocks] per block: sum q, sum q^2, max |q|
    void* rho = nullptr;       // [ncell] mesh charge of type R (FP32 in the mixed form), FFT input
    float* box = nullptr;      // push form of make_rho: [ntiles][box points] FP32 partial sums
    size_t box_bytes = 0;      // bytes of box
    bool spread_push = false;  // make_rho in the push form (mixed form, P = 7, box within the LDS)
    int spread_mode = 0;       // 0: by order, 1: owner-computes form only, 2: push form whenever it fits
    void* rho_hat = nullptr;   // [nspec] complex R
    void* spec = nullptr;      // [(ncomp + 1) * nspec] complex R: field spectra, then phi spectrum
    void* field = nullptr;     // [(ncomp + 1) * ncell] R: field meshes, then phi (ik adjoint)
    double* G = nullptr;       // [nspec] (C / V) G(k); own transforms: [Kz/2+1][Ky/2+1][Kx/2+1] octant
    double* epart = nullptr;   // [kspace blocks] partial sums of the mesh energy
    double* eterms = nullptr;  // [10] E, E_mesh, E_self, E_bg, Q, sum q^2, then from the particle map:
                               // max count, max |q|, sum q^2, unused
    void* wtab = nullptr;      // stencil-weight table (PPPM_FLAG_WEIGHT_TABLE)
    double* sfc = nullptr;     // (PPPM_FLAG_AD_SELF_FORCE) [6 + 6 * kspace blocks]: per axis
                               // (-1)^P 2 pi S1_d / h_d, then 4 pi S2_d / h_d (factors of the sines
                               // of the stencil fraction); block partials after them
    int* flags = nullptr;      // [1] sticky non-finite flag
    void* fft_work = nullptr;
    size_t fft_work_bytes = 0;
    int64_t qpart_blocks = 0;
    int* hist = nullptr;       // [HIST_MAX_BLOCKS * nbins] (histogram form) per-block bin counts,
                               // then per-block offsets within each bin
    int hist_blocks = 0;       // blocks of the last histogram map
    int hist_chunk = 0;        // charges per block of the last histogram map
    int64_t epart_blocks = 0;

    // Poisson step: the library's own LDS transforms (power-of-two meshes)
    // or rocFFT plans (other sizes)
    bool own_fft = false;
    void* fft_tw = nullptr;    // [Kx + Ky + Kz] complex R twiddle tables (own transforms)
    int fx_rows = 1;           // rows per block of the x passes
    int fy_xc = 1, fz_xc = 1;  // x columns per block of the y and z passes
    int fz_blocks = 0;         // blocks of the z pass (energy partial sums)
    int fft_pitch = 0;         // row pitch of the own transforms' spectra (complex values)
    bool fft_xy = false;       // x and y passes fused per z plane (mixed form, plane fits in LDS)
    int64_t spec_len = 0;      // elements of one spectrum: nspec (rocFFT) or Kz Ky fft_pitch (own)
    rocfft_plan fft_fwd = nullptr;   // D2Z of rho
    rocfft_plan fft_inv = nullptr;   // C2R batch ncomp
    rocfft_plan fft_inv1 = nullptr;  // C2R batch 1 (phi of an ik plan)
    rocfft_execution_info fft_info = nullptr;

    // launch geometry
    pppm::LaunchCfg spread_cfg{}, gather_cfg{}, adjoint_cfg{};

    // state
    pppm::Stage stage = pppm::Stage::Empty;
    int64_t n = 0;
    const void* pos_ptr = nullptr;
    const void* q_ptr = nullptr;
    bool phi_valid = false;  // field buffer holds phi for the adjoint

    std::string last_error;
};

namespace pppm {

// ---- host launchers (each returns hipGetLastError() of its launches) ----
hipError_t launch_map_count(pppm_plan_s* pl, int64_t n, const void* pos, const void* q);
hipError_t launch_scan(pppm_plan_s* pl);
hipError_t launch_scatter(pppm_plan_s* pl, int64_t n, const void* pos, const void* q);
hipError_t launch_spread(pppm_plan_s* pl, double* rho_user);
hipError_t launch_gather(pppm_plan_s* pl, int mode, void* out0, void* out1, const double* grad_energy);
hipError_t launch_influence(pppm_plan_s* pl);
hipError_t launch_self_force_coef(pppm_plan_s* pl);
int kspace_blocks(long long nspec);
hipError_t launch_kspace(pppm_plan_s* pl, bool phi_only);
hipError_t launch_energy_final(pppm_plan_s* pl, double* energy_out);
EnergySums energy_sums(const pppm_plan_s* pl, double* energy_out);
hipError_t launch_copy_terms(pppm_plan_s* pl, double* out3);
bool own_fft_supported(const int K[3], bool mixed);
void own_fft_shapes(pppm_plan_s* pl);
bool own_fft_shapes_ok(const pppm_plan_s* pl);
size_t own_fft_lds_max(const pppm_plan_s* pl);
hipError_t launch_own_fft_twiddles(pppm_plan_s* pl);
// phi_only false: the forward Poisson step, whose last pass also takes the
// final energy sums (into the plan's terms and, if not null, energy_out).
hipError_t launch_own_poisson(pppm_plan_s* pl, bool phi_only, double* energy_out);

// LDS bytes a kernel needs for the plan's tile shape.
size_t spread_lds_bytes(const MapGeo& g);
size_t spread_push_lds_bytes(const MapGeo& g);
int64_t spread_box_points(const MapGeo& g);
size_t gather_lds_bytes(const MapGeo& g, int order, int ncomp, size_t elem_bytes, int threads);
size_t gather_field_lds_bytes(const MapGeo& g, int order, int ncomp, size_t elem_bytes);

enum GatherMode { GATHER_IK = 0, GATHER_AD = 1, GATHER_ADJOINT = 2 };

}  // namespace pppm
