/*
 * pppm.h - C ABI of the MI355X (gfx950) PPPM particle-mesh library
 *          (libpppm_mi355x.so).
 *
 * The library computes the long-range half of the Ewald split of the Coulomb
 * sum with the particle-particle particle-mesh method (paper Section 2.1):
 *   1. particle map: each charge's mesh coordinate, stencil start and
 *      fraction (the "calculation of stencil coefficients", Section 3.1);
 *   2. make_rho (the paper's Map-Charge): spread q times the order-P stencil
 *      coefficients onto a periodic mesh;
 *   3. Poisson solve in k-space by FFT (Equation 2; Section 3.2): the
 *      library's own transform kernels when every mesh size is a power of
 *      two (8..1024 in the mixed form, 8..256 in FP64) or, in the mixed
 *      form, 2^a m with m in {3, 5, 7, 9} up to 448 (K_x / 2 from the same
 *      list), rocFFT otherwise, with the influence-function multiply and
 *      energy sums in between;
 *   4. fieldforce (the paper's Distribute-Force): gather the three field
 *      meshes (ik) or the derivative-weighted potential (ad) back to forces
 *      F_j = -q_j grad Phi (Equation 3).
 * plus the mesh energy and its adjoint (gradients of the energy with respect
 * to positions and charges).
 *
 * Conventions
 *   - Orthorhombic periodic box [lo, lo + L) per axis; mesh K_d points per
 *     axis, grid point m at lo + m h, h = L / K.  Positions anywhere finite
 *     are wrapped periodically.
 *   - Stencil order P in [2, 7]: the stencil coefficients of one axis are the
 *     order-P cardinal B-spline (degree P - 1) evaluated at the charge's
 *     offset from the P mesh points starting at s = floor(u + 1 - P/2),
 *     u = (x - lo)/h.
 *   - Energy E = E_mesh + E_self + E_bg in FP64:
 *       E_mesh = (C / 2V) sum_k G(k) |rho_hat(k)|^2,
 *       E_self = -C g / sqrt(pi) sum q_i^2,  E_bg = -C pi Q^2 / (2 V g^2).
 *     G is the optimal influence function of the chosen differentiation mode.
 *   - rho is charge per mesh point (sum rho = sum q), FP64, C order
 *     [Kz][Ky][Kx] (x fastest).
 *   - pos, forces, grad_pos: N x 3 row-major (x, y, z per particle); q and
 *     grad_q: N.  All in the caller's particle order and of params.io_dtype.
 *
 * Memory and streams
 *   - Every array argument of an enqueueing call is a DEVICE pointer owned by
 *     the caller.  The library reads or writes it only during the enqueued
 *     work and never frees or retains it.
 *   - A plan owns its scratch (binned particle records, permutation, meshes,
 *     influence function, transform tables or rocFFT plans and work buffers)
 *     and frees it in pppm_plan_destroy.
 *   - All work is enqueued on the HIP stream given at plan creation; calls
 *     return when the work is enqueued.  Results are valid after the stream
 *     is synchronised (or pppm_sync).  One plan per stream; calls on one plan
 *     are not thread-safe.
 *
 * Errors
 *   Every call returns a pppm_status; PPPM_OK is 0, errors are negative.  A
 *   failed call enqueues nothing further; details are in pppm_last_error.
 *   Non-finite inputs are detected on the device when PPPM_FLAG_CHECK_FINITE
 *   is set; the sticky flag is reported by pppm_sync.  Without the flag a
 *   non-finite coordinate is treated as 0 so that all mesh accesses stay in
 *   bounds, and the results for that particle are meaningless.
 */
#ifndef PPPM_MI355X_H
#define PPPM_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pppm_plan_s *pppm_plan;

typedef enum {
    PPPM_OK = 0,
    PPPM_ERR_ARG = -1,       /* null pointer, n < 0, n > max_particles, L <= 0, g <= 0, C == 0, ... */
    PPPM_ERR_ORDER = -2,     /* P outside [2, 7] */
    PPPM_ERR_MESH = -3,      /* K_d < P, K_d < 2, K_d > 2048 or more than 2^30 mesh points */
    PPPM_ERR_DTYPE = -4,     /* unknown precision or io dtype */
    PPPM_ERR_NONFINITE = -5, /* a position or charge was NaN/Inf (checked mode, at pppm_sync) */
    PPPM_ERR_OOM = -6,       /* device allocation failed */
    PPPM_ERR_HIP = -7,       /* a HIP runtime call or kernel launch failed */
    PPPM_ERR_FFT = -8,       /* rocFFT plan creation or execution failed */
    PPPM_ERR_STATE = -9      /* call out of order (e.g. backward without a matching forward) */
} pppm_status;

/* Differentiation mode (Section 2.1): ik = gradient in k-space, three field
 * meshes gathered; ad = analytic gradient of the interpolated potential. */
typedef enum { PPPM_DIFF_IK = 0, PPPM_DIFF_AD = 1 } pppm_diff;

/* Arithmetic of the particle-mesh steps.
 *   FP64:  every step in double precision.
 *   MIXED: stencil weights and their products in FP32, rounded without
 *          bias to a fixed-point unit and summed exactly in LDS (32-bit sums;
 *          64-bit in tiles that read more than 8,192 charges or where more
 *          than 512 charges can reach one point, and in every tile when the
 *          largest |q| exceeds 8 times the RMS |q|); each mesh point
 *          is flushed as FP64 (the caller's rho) and as FP32 (the plan's FFT
 *          input); FFTs, field meshes and gathers in FP32; the energy
 *          reduction in FP64. */
typedef enum { PPPM_PREC_FP64 = 0, PPPM_PREC_MIXED = 1 } pppm_prec;

/* Element type of the particle-side arrays (pos, q, forces, gradients). */
typedef enum { PPPM_F32 = 0, PPPM_F64 = 1 } pppm_dtype;

#define PPPM_FLAG_CHECK_FINITE 1u
/* Stencil weights from a table instead of their polynomials: the variant the
 * paper describes for its mapping functions (Section 3.1), T + 1 entries per
 * weight at the fractions i / T, the nearest entry used.  An approximation
 * whose error falls as 1 / T.  T is given in flag bits 8..23 by
 * PPPM_WEIGHT_TABLE_SIZE(T), 16 <= T <= 65535; 0 there means T = 5000. */
#define PPPM_FLAG_WEIGHT_TABLE 2u
#define PPPM_WEIGHT_TABLE_SIZE(T) (((uint32_t)(T) & 0xFFFFu) << 8)
/* ad only (PPPM_ERR_ARG with ik): subtract from each ad force the charge's
 * self-force, the force its own mesh charge exerts on it.  With ad the
 * gradient of the interpolated potential is not symmetric between a charge
 * and its own stencil (Section 2.1's ad mode), so a lone charge feels a force
 * that is periodic in its position within a mesh cell.  It is removed to its
 * leading harmonics, per axis
 *   F_self,d = q^2 / h_d [2 pi S1_d sin(2 pi u_d) + 4 pi S2_d sin(4 pi u_d)],
 * u = (x - lo) / h, S1_d / S2_d the sums over the spectrum of (C/V) G times
 * the B-spline transform products of aliases one and two apart along d
 * (computed once at plan creation).  The forces are then no longer the exact
 * gradient of the energy; the energy and pppm_energy_backward are unchanged. */
#define PPPM_FLAG_AD_SELF_FORCE 4u

typedef struct {
    double box_lo[3];      /* lower corner of the periodic box */
    double box_len[3];     /* edge lengths L_d > 0 */
    int32_t mesh[3];       /* K_x, K_y, K_z */
    int32_t order;         /* stencil order P in [2, 7] */
    double g_ewald;        /* Ewald splitting parameter g > 0 (1/length) */
    double coulomb_c;      /* Coulomb constant C != 0 (energy * length / charge^2) */
    pppm_diff diff;
    pppm_prec prec;
    pppm_dtype io_dtype;
    int64_t max_particles; /* capacity; 0 <= n <= max_particles <= 2^31 - 1 */
    uint32_t flags;        /* PPPM_FLAG_* */
} pppm_params;

/* Check a parameter set without touching the GPU.  Pure host function. */
pppm_status pppm_validate(const pppm_params *params);

/* Create a plan: validates params, allocates device scratch, builds the
 * influence function and the transform tables or rocFFT plans.  hip_stream is
 * a hipStream_t (NULL = the default stream) on the current device.  On
 * success *out is a plan.
 * make_rho (Map-Charge, Section 3.1) runs in one of two forms with the same
 * results to the fixed-point resolution: each mesh tile pulling the charges
 * whose stencils reach it, or, in the mixed precision, each tile pushing its
 * own charges' whole stencils into an extended box that a second kernel
 * folds into the mesh.  The mixed precision takes the push form at P >= 6,
 * and at P = 5 when there are fewer mesh tiles than compute units.
 * PPPM_SPREAD=visit or =push in the environment when the plan is
 * created forces one form (push only in the mixed precision and where its
 * box fits the device's LDS). */
pppm_status pppm_plan_create(const pppm_params *params, void *hip_stream, pppm_plan *out);

/* Release a plan and all its device memory.  Synchronises its stream first.
 * NULL is accepted and ignored. */
pppm_status pppm_plan_destroy(pppm_plan plan);

/* Step 1 - particle map (Section 3.1): wrap each position into the box,
 * compute its stencil start and fraction per axis, bin the particles by mesh
 * sub-brick and store them in binned order for the steps that follow.
 * pos: N x 3, q: N, device, io_dtype.  n may be 0. */
pppm_status pppm_particle_map(pppm_plan plan, int64_t n, const void *pos, const void *q);

/* Step 2 - make_rho (Map-Charge, Section 3.1): spread the mapped charges onto
 * the plan's mesh.  If rho is not NULL the mesh charge is also written to
 * rho (device, FP64, Kz*Ky*Kx).  Requires pppm_particle_map. */
pppm_status pppm_make_rho(pppm_plan plan, double *rho);

/* Step 3 - Poisson solve (Equation 2; Section 3.2): FFT of the mesh charge,
 * influence-function multiply, energy reduction, inverse FFT(s) to the field
 * meshes (ik: three) or the potential mesh (ad: one).  If energy is not NULL
 * the total energy E (one FP64 on the device) is written there.
 * Requires pppm_make_rho. */
pppm_status pppm_poisson(pppm_plan plan, double *energy);

/* Step 4 - fieldforce (Distribute-Force, Section 3.1): gather the field
 * meshes back to per-particle forces (device, N x 3, io_dtype, caller order).
 * Requires pppm_poisson. */
pppm_status pppm_fieldforce(pppm_plan plan, void *forces);

/* Steps 1-4 in one call.  rho, energy and forces may each be NULL (forces
 * NULL skips the gather).  Same layouts as above. */
pppm_status pppm_compute(pppm_plan plan, int64_t n, const void *pos, const void *q,
                         double *rho, double *energy, void *forces);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid hipMalloc): steps 1-4 as
 * pppm_compute from the parameters alone, with no plan.  Every buffer of the
 * transient plan (binned charges, meshes, spectra, influence function,
 * transform tables) is carved from one static device array of
 * PPPM_NOALLOC_SCRATCH_BYTES per GPU, which the library holds for the life
 * of the process; the call allocates nothing and launches no memset (what
 * must start at zero is cleared by a kernel), so it can be captured.
 * The influence function and transform tables are rebuilt by every call (at
 * 128^3 they take about 0.1 ms).  Same arguments, layouts and results as
 * pppm_compute; hip_stream as in pppm_plan_create.  Where a plan would take
 * the push form of make_rho and its boxes do not fit the array beside the
 * rest, the call takes the owner-computes form: its results then agree with
 * pppm_compute to the fixed-point resolution rather than bit for bit.
 * Limits: the mesh must be one the library's own transforms take (see the
 * Poisson step above; rocFFT plans allocate), and neither
 * PPPM_FLAG_WEIGHT_TABLE nor PPPM_FLAG_CHECK_FINITE is taken; parameters that
 * need more scratch than the array holds (about max_particles * 44 bytes plus
 * 20 to 40 bytes per mesh point) return PPPM_ERR_ARG, others as
 * pppm_plan_create and pppm_compute.  Errors are reported through
 * pppm_last_error(NULL).
 * Every call on one GPU shares that GPU's array and it keeps the last call's
 * contents: calls that overlap on one GPU (other streams, other threads)
 * race; order them on one stream or synchronise between them. */
#define PPPM_NOALLOC_SCRATCH_BYTES ((size_t)96 << 20)
pppm_status pppm_compute_noalloc(const pppm_params *params, void *hip_stream, int64_t n, const void *pos,
                                 const void *q, double *rho, double *energy, void *forces);

/* Adjoint of the energy.  Given grad_energy (one FP64 on the device, dL/dE),
 * writes grad_pos = dL/dE * dE/dr_i (N x 3) and grad_q = dL/dE * dE/dq_i (N),
 * device, io_dtype, caller order:
 *   dE/dq_i = phi(r_i) - 2 C g q_i / sqrt(pi) - C pi Q / (V g^2),
 *   dE/dr_i = q_i grad phi(r_i),
 * with phi the mesh potential of the plan's influence function, interpolated
 * with the same stencil.  Uses the mesh kept by the last pppm_compute (or
 * pppm_poisson), which must have been called with the same pos, q and n
 * pointers and count (else PPPM_ERR_STATE), and the charges binned by that
 * call: the stencil weights are recomputed from the binned positions of the
 * forward step, so the gradient belongs to the positions the potential was
 * computed for.  Either output may be NULL. */
pppm_status pppm_energy_backward(pppm_plan plan, const double *grad_energy, int64_t n,
                                 const void *pos, const void *q, void *grad_pos, void *grad_q);

/* Copy the three energy terms (E_mesh, E_self, E_bg) of the last Poisson
 * solve to out3 (device, 3 FP64).  Enqueued on the plan's stream. */
pppm_status pppm_energy_terms(pppm_plan plan, double *out3);

/* Synchronise the plan's stream and report deferred errors: a HIP error, or
 * PPPM_ERR_NONFINITE when checking is on and a non-finite input was seen
 * (the flag is cleared by this call). */
pppm_status pppm_sync(pppm_plan plan);

/* Static description of a status code. */
const char *pppm_status_string(pppm_status status);

/* Detail of the last error on this plan ("" if none).  The string stays
 * valid until the next call on the plan.  NULL plan: last error of
 * pppm_validate / pppm_plan_create on the calling thread. */
const char *pppm_last_error(pppm_plan plan);

/* Launch geometry, for tuning.  tile[3] = mesh points per workgroup tile
 * along x, y, z (each in [1, 64]; an edge at least the mesh size makes one
 * tile along that axis); the tile shape is shared by the
 * binning, spread and gather kernels of the plan, so changing it discards the
 * mapped particles (call pppm_particle_map or pppm_compute again).  Every
 * tile must be at least order - 1 points thick along an axis that has more
 * than one tile.  threads = workgroup size of the kernel `which`, a multiple
 * of 64: 0 = spread (64..1024), 1 = gather, forward (64..512; the mixed ik
 * gather 64..1024, by default 768 where the tile's LDS allows), 2 = gather,
 * adjoint (64..512).  A new tile that leaves no room for the forward
 * gather's workgroup narrows it to the widest that fits.
 * Returns PPPM_ERR_ARG (and changes nothing) for an unusable geometry,
 * including one whose shared memory exceeds the device limit. */
pppm_status pppm_plan_set_launch(pppm_plan plan, int32_t which, const int32_t *tile, int32_t threads);

/* Current launch geometry (see pppm_plan_set_launch); host pointers. */
pppm_status pppm_plan_get_launch(pppm_plan plan, int32_t which, int32_t *tile, int32_t *threads);

#ifdef __cplusplus
}
#endif

#endif /* PPPM_MI355X_H */
