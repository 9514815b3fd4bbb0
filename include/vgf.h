/*
 * vgf.h -- C ABI of the MI355X (gfx950) free-space Poisson solver library
 * libvgf.so: the Vico-Greengard-Ferrando (VGF) method and, beside it, the
 * Hockney-Eastwood (HE) method, as compared in Zou, Kim & Cerfon,
 * arXiv:2103.08531.
 *
 * Problem (Sec. I, Eq. 1): Laplace(phi) = -rho in free space, E = -grad(phi),
 * for rho sampled on a uniform grid of n_a points with spacing h_a per axis
 * (Sec. I, the text around Eq. 3). The solution is the convolution of rho
 * with the free-space Green's function (Eq. 2):
 *   HE : with the trapezoidal rule and the kernel h^d G(|n h|), its origin
 *        value regularised (Eq. 3 and the sentence after it);
 *   VGF: with the kernel obtained once per grid as the inverse DFT, on the
 *        (4N)^d oversampled grid, of the closed-form spectrum of the kernel
 *        truncated at radius L (Eqs. 4-8), restricted to offsets |n_a| < N_a
 *        (Sec. II, last paragraph).
 * Each solve is then an aperiodic convolution computed with FFTs on the
 * zero-padded (2N)^d grid (Eq. 3); the field is obtained by Fourier
 * differentiation, i.e. multiplying by -i k_a before the inverse transform
 * (Sec. III.A), with the factor of the Nyquist wavenumber set to zero.
 *
 * Conventions common to every call:
 *  - Every status is a vgf_status; VGF_OK is 0, errors are negative. No C++
 *    exception crosses this interface and no call aborts the process.
 *  - rho, phi, E and gradient buffers are DEVICE pointers owned by the
 *    caller, C-contiguous with the last axis fastest, in the plan's precision
 *    (double for VGF_F64, float for VGF_F32). E is planar: E[a] starts at
 *    E + a * prod(n), a = 0..dim-1, and holds -d(phi)/dx_a.
 *  - Calls are asynchronous and stream-ordered on the stream passed in; none
 *    synchronises with the host except vgf_plan_create, vgf_plan_get_kernel
 *    and vgf_plan_get_spectrum, which do. A plan owns a workspace and must be
 *    used by one stream at a time; distinct plans are independent.
 *  - Supported sizes: every even n_a = 2^a 3^b (a >= 1) with
 *    8 <= n_a <= 512, i.e. n_a in {8, 12, 16, 18, 24, 32, 36, 48, 54, 64, 72,
 *    96, 108, 128, 144, 162, 192, 216, 256, 288, 324, 384, 432, 486, 512};
 *    2D plans in the default layout (no VGF_LAYOUT_AXIS0) also take
 *    n_a in {576, 648, 768, 864, 972, 1024}, i.e. every even 2^a 3^b up to
 *    1024 (the padded length 2 n_a is an FFT length of radices 8, 4, 2 and 3
 *    that the library instantiates). Other sizes, odd ones included, return
 *    VGF_ERR_UNSUPPORTED_SIZE.
 */
#ifndef VGF_H
#define VGF_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vgf_plan_s* vgf_plan;

typedef enum {
  VGF_OK = 0,
  VGF_ERR_INVALID_ARG = -1,      /* null pointer, bad dim/method/precision/flags */
  VGF_ERR_UNSUPPORTED_SIZE = -2, /* an n_a outside the supported set */
  VGF_ERR_L_WINDOW = -3,         /* L outside (diameter, min_a(4 n_a h_a - extent_a)) */
  VGF_ERR_OUT_OF_MEMORY = -4,    /* device allocation failed or exceeds VGF_MAX_WORKSPACE */
  VGF_ERR_HIP = -5,              /* a HIP runtime call failed (see vgf_plan_hip_error) */
  VGF_ERR_NOT_REQUESTED = -6,    /* an output that the plan was not created for */
  VGF_ERR_SCRATCH_LIMIT = -7     /* vgf_solve_noalloc: the plan's workspace exceeds its scratch */
} vgf_status;

/* VGF: Vico-Greengard-Ferrando (Sec. II). HE: Hockney-Eastwood (Eq. 3) with
 * the origin weight vol * G0, G0 = 1/(4 pi) in 3D, 1/(2 pi) in 2D (the
 * singular factor replaced by 1). HE_NEARBY: origin weight vol * G(r0) at
 * r0 = half the smallest spacing ("nearby value" of the comparison figures,
 * Sec. III.A). HE_CELLAVG: origin weight = the integral of G over the cell
 * prod_a [-h_a/2, h_a/2] ("cell average"). All HE variants share w[n] =
 * vol * G(|n h|) for n != 0, vol = prod_a h_a. */
typedef enum {
  VGF_METHOD_VGF = 0,
  VGF_METHOD_HE = 1,
  VGF_METHOD_HE_NEARBY = 2,
  VGF_METHOD_HE_CELLAVG = 3
} vgf_method;
typedef enum { VGF_F64 = 0, VGF_F32 = 1 } vgf_precision;
/* Outputs a plan may return, and how E is obtained:
 *   VGF_OUT_PHI, VGF_OUT_E : the fields later solves may return;
 *   VGF_FIELD_CENTERED     : (with VGF_OUT_E) E = -D phi by second-order
 *     finite differences of the computed phi -- centred at interior points,
 *     one-sided (-3, 4, -1)/(2h) on the first and (3, -4, 1)/(2h) on the last
 *     plane of each axis -- instead of Fourier differentiation. This is the
 *     "Finite Diff" field of the comparison figures (Sec. III.A); Fourier
 *     differentiation is the default. */
/*   VGF_FIELD_GRADIENT_KERNEL : (VGF method, with VGF_OUT_E) E_a = w_a * rho
 *     with w_a the gradient kernel: the inverse DFT on the 4N-oversampled grid
 *     of -i k_a times the windowed spectrum, restricted like the potential's
 *     kernel (Sec. II, applied to the field; the other reading of Sec. III.A's
 *     "multiplying by the wavevector"). The plan stores dim more kernel
 *     spectra; the multiply pass multiplies every field by its own spectrum
 *     and each field is inverted separately. */
/*   VGF_LAYOUT_AXIS0 : run the spectral multiply inside the axis-0 pass
 *     (real-to-complex along the last axis, strided axis-0 multiply pass)
 *     instead of the default (real-to-complex along axis 0, multiply pass
 *     along the contiguous last axis). Both compute the same discrete
 *     result, for every field mode. */
enum {
  VGF_OUT_PHI = 1u,
  VGF_OUT_E = 2u,
  VGF_FIELD_CENTERED = 16u,
  VGF_FIELD_GRADIENT_KERNEL = 32u,
  VGF_LAYOUT_AXIS0 = 64u
};

/* Build a plan for a fixed grid (Sec. II: one precomputation per grid, then
 * a solve per right-hand side).
 *   out      : receives the plan handle (host pointer, not null).
 *   dim      : 2 or 3.
 *   n[dim]   : points per axis (host array).
 *   h[dim]   : grid spacing per axis, > 0 (host array).
 *   method   : a vgf_method (VGF, or one of the HE variants).
 *   prec     : arithmetic and buffer type of every solve. The kernel spectrum
 *              is always computed in FP64 and, for VGF_F32, rounded to FP32
 *              once; FFT twiddles are FP64 values rounded to the plan type.
 *   L        : truncation radius of the VGF kernel (Eq. 4). L <= 0 selects
 *              1.1 x the box diameter; a NaN or infinite L is rejected with
 *              L_WINDOW. Must lie strictly inside
 *              (diameter, min_a(4 n_a h_a - (n_a - 1) h_a)): below it the
 *              truncated kernel misses source-target pairs (Sec. II), above
 *              it the 4N-periodic images reach the box. Ignored for HE.
 *   outputs  : VGF_OUT_PHI | VGF_OUT_E, the fields later solves may return,
 *              optionally | VGF_FIELD_CENTERED or | VGF_FIELD_GRADIENT_KERNEL
 *              (either requires VGF_OUT_E; the latter the VGF method), and
 *              optionally | VGF_LAYOUT_AXIS0.
 *   stream   : stream on which the FP64 precompute runs; the call
 *              synchronises it before returning.
 * Environment, read here: VGF_STREAM_MIN_BYTES (default 33554432): forward
 * solves in the default layout whose input (rho of all entries of a launch)
 * has at least this many bytes use non-temporal loads and stores in their
 * middle passes; VGF_TILED_Y=0: 3D forward solves in the default layout keep
 * the multiply pass's output in plain rows instead of the axis-1 inverse's
 * tile order. Results are identical either way, only speed differs.
 * Errors: INVALID_ARG, UNSUPPORTED_SIZE, L_WINDOW, OUT_OF_MEMORY, HIP. On
 * error *out is set to NULL and nothing is leaked. */
vgf_status vgf_plan_create(vgf_plan* out, int dim, const int64_t* n, const double* h,
                           vgf_method method, vgf_precision prec, double L,
                           unsigned outputs, hipStream_t stream);

/* One solve (the per-right-hand-side path of Sec. II / Eq. 3):
 *   rho : device input, prod(n) values.
 *   phi : device output, prod(n) values, or NULL to skip the potential.
 *   E   : device output, dim * prod(n) values (planar), or NULL.
 * Requesting a field the plan was not created for returns NOT_REQUESTED;
 * phi == E == NULL returns INVALID_ARG. Enqueued on `stream`. */
vgf_status vgf_solve(vgf_plan plan, const void* rho, void* phi, void* E, hipStream_t stream);

/* vgf_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same passes and the same results as vgf_solve, bit for bit, but the solve
 * workspace is a static device array of VGF_NOALLOC_SCRATCH_BYTES (64 MiB)
 * that every device the library runs on holds until the process ends,
 * instead of the plan's workspace. The call itself allocates nothing (no
 * hipMalloc, hipFree or allocating library routine); the plan's kernel
 * spectra and twiddles come from vgf_plan_create as usual.
 *   plan, rho, phi, E, stream : as for vgf_solve (device buffers owned by the
 *   caller; the current device must be the plan's).
 * The scratch is shared by every call on one device and keeps the last
 * call's contents (nothing in it needs to start at zero): calls that overlap
 * on one device -- on different streams, or from different threads --
 * race, and must be ordered by the caller.
 * Errors: as vgf_solve, and SCRATCH_LIMIT when vgf_plan_workspace_bytes of
 * the plan exceeds the scratch (e.g. 3D grids above about 64^3 in FP64 or
 * 90^3 in FP32); nothing is enqueued then. */
#define VGF_NOALLOC_SCRATCH_BYTES (64u << 20)
vgf_status vgf_solve_noalloc(vgf_plan plan, const void* rho, void* phi, void* E, hipStream_t stream);

/* Adjoint of vgf_solve (for reverse-mode differentiation):
 *   g_rho = K^T g_phi + sum_a K_a^T g_E[a],
 * where K maps rho to phi and K_a maps rho to E[a]. g_phi or g_E may be NULL
 * (treated as zero), not both. All buffers are device buffers shaped like the
 * corresponding forward outputs / input. Enqueued on `stream`. */
vgf_status vgf_solve_adjoint(vgf_plan plan, const void* g_phi, const void* g_E, void* g_rho,
                             hipStream_t stream);

/* Many independent solves, possibly on different plans (grids), enqueued one
 * after another, each exactly as vgf_solve: rho[i], phi[i], E[i] follow
 * vgf_solve for plans[i] (phi and E arrays may be NULL, or hold NULL
 * entries). The same plan may appear more than once: its solves are then
 * serialised on its workspace. Enqueued on `stream`; on the first invalid
 * entry nothing is enqueued. (vgf_batch_* below runs the same solves with one
 * launch per pass and per grid, and as one captured graph.) */
vgf_status vgf_solve_batched(const vgf_plan* plans, int count, const void* const* rho,
                             void* const* phi, void* const* E, hipStream_t stream);

/* ---- Batches: one precompute per grid, then many right-hand sides per call
 * (Sec. II: the kernel spectrum is computed once per grid and reused for
 * every density; Eq. 3 is applied to each right-hand side independently). ----
 *
 * A batch fixes, at creation, the plan of each of its `count` entries;
 * entries may use different plans (grids of uneven size, either precision).
 * Entries sharing a plan handle form a group: every pass of a group is one
 * launch over all of its entries, each entry with its own workspace (owned
 * by the batch), so the group's entries run concurrently. Groups are
 * independent. With VGF_BATCH_GRAPH the first vgf_batch_solve (and any
 * later one that asks for a different set of outputs) captures all launches
 * into one hipGraph, the groups as parallel branches, and every solve
 * replays it with one graph launch on `stream`.
 *
 * The plans must outlive the batch. A batch, like a plan, serves one stream at
 * a time (its workspaces are shared by its solves); batches do not use the
 * plans' own workspaces, so plans stay usable for vgf_solve meanwhile on the
 * same stream. Memory: vgf_batch_workspace_bytes. */
typedef struct vgf_batch_s* vgf_batch;
enum { VGF_BATCH_GRAPH = 1u };

/* plans[0..count): the plan of each entry (non-NULL, count >= 1; any method,
 * precision, layout and field mode). A group of a VGF_FIELD_CENTERED plan
 * runs its passes for phi over all entries, then the difference field over
 * all entries in one more launch (phi goes to the entry's workspace when
 * only E is asked for). flags: 0 or VGF_BATCH_GRAPH. Allocates the group
 * workspaces (VGF_ERR_OUT_OF_MEMORY beyond VGF_MAX_WORKSPACE). Enqueues
 * nothing. */
vgf_status vgf_batch_create(vgf_batch* out, const vgf_plan* plans, int count, unsigned flags);

/* Solves every entry i: rho[i] -> phi[i], E[i], with the layout, dtype and
 * output rules of vgf_solve for the entry's plan. phi (or E) is either NULL,
 * meaning no entry gets that output, or holds a non-NULL buffer for every
 * entry (VGF_ERR_INVALID_ARG otherwise); at least one of them is non-NULL.
 * Pointers may differ from call to call: the batch refreshes its device
 * pointer tables on `stream` (a small kernel, no host staging) before the
 * passes when they change. Stream-ordered and asynchronous; nothing is
 * enqueued when an argument is invalid. Results equal vgf_solve's bit for bit
 * (same kernels, same arithmetic order). */
vgf_status vgf_batch_solve(vgf_batch batch, const void* const* rho, void* const* phi, void* const* E,
                           hipStream_t stream);

/* Adjoint of every entry i (the transpose of the per-right-hand-side
 * convolution of Sec. II / Eq. 3 and of its field, Sec. III.A):
 * g_rho[i] = K^T g_phi[i] + sum_a K_a^T g_E[i][a], with the arguments and
 * rules of vgf_solve_adjoint for the entry's plan.
 * g_rho holds a non-NULL buffer for every entry; g_phi (or g_E) is NULL
 * (that cotangent is zero for every entry) or holds a non-NULL buffer for
 * every entry; at least one of them is non-NULL (VGF_ERR_INVALID_ARG
 * otherwise; VGF_ERR_NOT_REQUESTED for a cotangent of an output the entry's
 * plan was not created for). Groups of default-layout plans with Fourier
 * fields run each pass as one launch over all of their entries; the other
 * groups run one vgf_solve_adjoint per entry (on the plan's own workspace).
 * Always direct launches on `stream` (a captured graph replays solves only);
 * stream-ordered and asynchronous; nothing is enqueued when an argument is
 * invalid. Results equal vgf_solve_adjoint's bit for bit. */
vgf_status vgf_batch_adjoint(vgf_batch batch, const void* const* g_phi, const void* const* g_E,
                             void* const* g_rho, hipStream_t stream);

/* Tunes every group's schedule as vgf_plan_autotune does, with the group's
 * entry count per launch (a schedule that suits one grid alone may not suit
 * many at once), on the caller's buffers (arguments as vgf_batch_solve;
 * outputs receive results). Cached per process per (grid, precision,
 * outputs, entries). Groups start with their plan's schedule; a captured
 * graph is dropped and recaptured by the next solve. Synchronises `stream`. */
vgf_status vgf_batch_autotune(vgf_batch batch, const void* const* rho, void* const* phi,
                              void* const* E, int reps, hipStream_t stream);

/* The schedule (int[5]) of group `group` (0 <= group < vgf_batch_groups). */
vgf_status vgf_batch_get_schedule(vgf_batch batch, int group, int* schedule);

/* Device bytes held by the batch (group workspaces and pointer tables). */
vgf_status vgf_batch_workspace_bytes(vgf_batch batch, size_t* bytes);

/* Number of groups (distinct plans, split further when a group would exceed
 * 65535 / (n0 + 1) entries); 0 for NULL. */
int vgf_batch_groups(vgf_batch batch);

/* The hipError_t behind the batch's last VGF_ERR_HIP. */
int vgf_batch_hip_error(vgf_batch batch);

/* Waits for nothing: destroy only after the batch's work has completed.
 * NULL is a no-op. */
void vgf_batch_destroy(vgf_batch batch);

/* ---- Tile schedules and their autotuner ----
 * The strided FFT passes come in two tile variants: 0 = one 128-byte row
 * segment of columns per workgroup (the default), 1 = half of it (more and
 * smaller workgroups). Strided are, in the default layout, the axis-0 R2C
 * and C2R passes and the axis-1 passes (3D); in the axis-0 layout
 * (VGF_LAYOUT_AXIS0) the axis-1 passes and the axis-0 multiply pass
 * (gradient-kernel plans: the axis-1 passes only). A variant changes only the launch shape: every line is
 * transformed with the same arithmetic, so results are bit-identical across
 * schedules. A schedule is an int[5], one value per pass in the order
 * VGF_PASS_R2C, VGF_PASS_C2C_FWD, VGF_PASS_FUSED, VGF_PASS_C2C_INV,
 * VGF_PASS_C2R. A value holds two bits: bit 0 is the variant of the pass's
 * first launch, bit 1 that of its later launches (the inverse passes launch
 * once per group of outputs, the two-output launch first; adjoints may
 * launch a pass more than once). In the default layout the multiply pass
 * along the contiguous axis (VGF_PASS_FUSED; not for gradient-kernel
 * plans, whose multiply pass has one schedule) has schedules too, its value
 * taken whole: bit 0 halves the lanes that share one line (twice the lines
 * per wavefront and the butterflies per lane), bit 1 lets each wavefront
 * walk 16 instead of 4 lines (fewer, longer workgroups); the walk is cut
 * where the grid would fall below 2048 workgroups. Passes without variants
 * (and the 2D middle passes, which do not exist) only take 0. */
enum { VGF_PASS_R2C = 0, VGF_PASS_C2C_FWD = 1, VGF_PASS_FUSED = 2, VGF_PASS_C2C_INV = 3,
       VGF_PASS_C2R = 4, VGF_NUM_PASSES = 5 };

/* Chooses the plan's schedule by measurement over four candidates (v = 0..3:
 * every strided pass at tile variant v & 1, the contiguous multiply pass at
 * value v): two warm-up solves per candidate, then `reps` rounds that each
 * run, per candidate, two solves of (rho, phi, E) (arguments as vgf_solve),
 * the second timed with HIP events after every launch on `stream`. For each
 * pass, its first launch and its later launches each take their fastest
 * repetition per value and keep the default unless another value is more
 * than 2% faster; a strided pass launched once gives both bits its first
 * launch's choice. A schedule so assembled
 * is kept only if it also beats the default on the whole solve by 1% (two
 * more solves per round and candidate). phi / E receive solve results.
 * Synchronises `stream`.
 * The choice is cached in the process per (grid, precision, outputs), so an
 * identical plan tuned again takes the cached schedule without running.
 * Errors: as vgf_solve, INVALID_ARG for reps <= 0. */
vgf_status vgf_plan_autotune(vgf_plan plan, const void* rho, void* phi, void* E, int reps,
                             hipStream_t stream);

/* The plan's schedule (int[5], see above); set checks every value (0..3)
 * and rejects a non-zero value for a pass that has no variants
 * (INVALID_ARG). */
vgf_status vgf_plan_get_schedule(vgf_plan plan, int* schedule);
vgf_status vgf_plan_set_schedule(vgf_plan plan, const int* schedule);

/* Gradient-kernel plans only (VGF_ERR_NOT_REQUESTED otherwise): the FP64
 * gradient kernel w_axis on [0, N)^d (odd in the axis, even in the others;
 * prod(n) doubles) and T_axis on [0, N]^d (the 2N spectrum of the odd
 * periodic kernel is -i T_axis; prod(n_a + 1) doubles). Synchronous. */
vgf_status vgf_plan_get_gradient_kernel(vgf_plan plan, int axis, double* host_out);
vgf_status vgf_plan_get_gradient_spectrum(vgf_plan plan, int axis, double* host_out);

/* The truncation radius the plan uses (0 for HE). */
vgf_status vgf_plan_get_L(vgf_plan plan, double* L);

/* Device bytes held by the plan (spectra, twiddles and solve workspace). */
vgf_status vgf_plan_workspace_bytes(vgf_plan plan, size_t* bytes);

/* Copies the FP64 restricted kernel w[n], n in [0,n_0) x ... (even octant;
 * the "numerical Green's function" of Sec. II, or the HE kernel) to the
 * host buffer `host_out` of prod(n) doubles. Synchronous. */
vgf_status vgf_plan_get_kernel(vgf_plan plan, double* host_out);

/* Copies the FP64 spectrum of the 2N-periodic kernel (real and even) on the
 * octant kappa in [0, n_0] x ... to `host_out` (prod(n_a + 1) doubles),
 * unscaled (DFT convention sum_n W[n] exp(-2 pi i kappa.n / 2N)).
 * Synchronous. */
vgf_status vgf_plan_get_spectrum(vgf_plan plan, double* host_out);

/* Per-launch timing (tracing support for benchmarks and profiling).
 * vgf_plan_profile_begin creates max_solves * (VGF_MAX_LAUNCHES + 1) HIP
 * events (host call, not stream-ordered); each following vgf_solve on this
 * plan, up to max_solves, records one event before its first launch and one
 * after each launch, on the solve's own stream. vgf_plan_profile_end waits
 * for the recorded events and writes, for each launch k of a solve, the mean
 * duration in milliseconds to launch_ms[k] and its pass (VGF_PASS_*) to
 * launch_pass[k]; the number of launches per solve to *nlaunch and the
 * number of timed solves to *nsolves; then destroys the events and stops
 * recording. Both arrays must hold VGF_MAX_LAUNCHES entries (unused ones are
 * 0 and -1). begin while already recording returns INVALID_ARG; end without
 * begin returns INVALID_ARG. */
enum { VGF_MAX_LAUNCHES = 16 };
vgf_status vgf_plan_profile_begin(vgf_plan plan, int max_solves);
vgf_status vgf_plan_profile_end(vgf_plan plan, double* launch_ms, int* launch_pass, int* nlaunch,
                                int* nsolves);

/* The last HIP error code recorded by a call on this plan (hipSuccess if
 * none). */
int vgf_plan_hip_error(vgf_plan plan);

void vgf_plan_destroy(vgf_plan plan);

/* Static, NUL-terminated description of a status code. */
const char* vgf_status_string(vgf_status status);

#ifdef __cplusplus
}
#endif
#endif /* VGF_H */
