/*
 * sce.h -- C ABI of the MI355X (gfx950) spectral canonical electrostatic
 * library: the per-step particle x mode sums of the gridless spectral
 * macroparticle method of Webb, "A Spectral Canonical Electrostatic
 * Algorithm" (arXiv:1508.07344), inside its symplectic leapfrog step.
 *
 * Model (periodic box [0, L)^3, V = L^3, permittivity eps0):
 *   modes      n in Z^3 with max_i |n_i| <= n_max and n != 0; k_n = 2 pi n / L.
 *              Mode spacing 2 pi / L keeps the box periodic (Section 8).
 *              The n = 0 mode is left out: a uniform neutralising background.
 *   half space H = { n_x > 0 } u { n_x = 0, n_y > 0 } u { n_x = n_y = 0, n_z > 0 }.
 *              Every mode pairs with its negative so the potential is real
 *              (Section 4); only H is stored, |H| = ((2 n_max + 1)^3 - 1) / 2.
 *              Canonical order: n_x = 0..n_max, then n_y = -n_max..n_max, then
 *              n_z = -n_max..n_max, skipping modes outside H.
 *   shape S(k) Fourier transform of the particle shape with S(0) = 1
 *              (Section 3): point 1, Gaussian exp(-|k|^2 a^2 / 2), or
 *              tent prod_d sinc^2(k_d a / 2).
 *   deposit    rho_n = S(k_n) sum_j q_j exp(-i k_n . x_j)
 *              (right-hand side of the discrete Poisson equation, Section 4).
 *   solve      phi_n = rho_n / (eps0 |k_n|^2): the delta field shape makes the
 *              k-squared matrix diagonal (Section 3, Section 4).
 *   force      F_j = -dW/dx_j = 2 q_j sum_{n in H} k_n Im(psi_n exp(i k_n . x_j)),
 *              psi_n = S(k_n) phi_n / V (the kick of the discrete
 *              Euler-Lagrange equations, Section 4).
 *   energy     W = (1 / (eps0 V)) sum_{n in H} |rho_n|^2 / |k_n|^2;
 *              kinetic K = 1/2 sum m |v|^2; total E = K + W.
 *   step       kick-drift-kick (default): v += (h/2) F/m, x = wrap(x + h v),
 *              F = F(x), v += (h/2) F/m, the end force reused by the next step;
 *              or drift-kick-drift, the velocity form the paper derives
 *              (Section 4): x = wrap(x + (h/2) v), F = F(x), v += h F/m,
 *              x = wrap(x + (h/2) v).  wrap(x) = x - L floor(x / L) in [0, L).
 *
 * Conventions for every entry point:
 *   - Returns sce_status: SCE_OK (0) or a negative error code.  No exception
 *     or signal crosses the ABI.  After an error, sce_last_error() holds a
 *     message.  SCE_EDEVICE (a HIP runtime error) leaves the context unusable.
 *   - A context is not thread-safe; distinct contexts are independent.
 *   - All device work is enqueued on the context's stream (its own, or the
 *     one given to sce_set_options).  Calls that return data to host memory
 *     synchronise that stream before returning.
 *   - Arrays of particle vectors are structure-of-arrays: [3][N] doubles
 *     (all x components, then all y, then all z).
 *   - on_device = 0: pointers are host memory, borrowed only for the call.
 *     on_device = 1: pointers are device memory on the context's device
 *     (for example a torch tensor's data_ptr()); they are borrowed until the
 *     call's work on the stream has finished (sce_sync).
 *   - The library owns every buffer it allocates and never frees caller memory.
 */
#ifndef SCE_H
#define SCE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SCE_OK = 0,
    SCE_EINVAL = -1,     /* bad argument (non-finite or out-of-range value, NULL pointer) */
    SCE_ENOMEM = -2,     /* device or host allocation failed */
    SCE_EDEVICE = -3,    /* HIP runtime error; the context is unusable afterwards */
    SCE_ESTATE = -4,     /* call made in the wrong state (e.g. no particles set) */
    SCE_ENOTSUP = -5,    /* unsupported option combination */
    SCE_EUNSTABLE = -6   /* non-finite energy found by sce_diagnostics */
} sce_status;

typedef enum { SCE_SHAPE_DELTA = 0, SCE_SHAPE_GAUSSIAN = 1, SCE_SHAPE_TENT = 2 } sce_shape_kind;

/* Arithmetic of the two particle x mode sums.  Positions, velocities, the
 * drift, the phase anchors, the cross-tile rho sums and the energy and
 * momentum reductions are FP64 in every mode. */
typedef enum {
    SCE_PREC_FP64 = 0,       /* FP64 phases, products and sums */
    SCE_PREC_FP32 = 1,       /* FP32 phase tables, FP32 products, FP32 sums within a particle tile */
    SCE_PREC_SPLIT_F16 = 2   /* FP16 hi+lo split products on the matrix cores, FP32 accumulation */
} sce_precision;

typedef enum { SCE_SCHEME_KDK = 0, SCE_SCHEME_DKD = 1 } sce_scheme;

/* Field shape Psi of the potential's modes (Section 3): delta functions (the
 * periodic box above) or tents of half-width dk (sce_create_tent). */
typedef enum { SCE_FIELD_DELTA = 0, SCE_FIELD_TENT = 1 } sce_field_kind;

typedef struct sce_ctx_s *sce_ctx;

/* Diagnostics at the current state (Section 6 reports energy and its kinetic,
 * capacitive and field parts, and the total momentum). */
typedef struct {
    int64_t step;              /* steps taken since the particles were set */
    double time;               /* sum of dt over those steps */
    double kinetic;            /* K = 1/2 sum m |v|^2 */
    double field;              /* W = (1/(eps0 V)) sum_H |rho|^2/|k|^2 at the current positions
                                  (tent fields: (eps0/2) phi^T K phi) */
    double field_self;         /* (sum q^2/(eps0 V)) sum_H S^2/|k|^2: constant self-energy within W
                                  (0 for tent fields, where it depends on the positions) */
    double interaction;        /* sum_j q_j Phi_j, Phi_j = 2 sum_H Re(psi e^{i k.x_j}); equals 2 W */
    double total;              /* K + W */
    double momentum[3];        /* sum m v */
    double momentum_abs_sum;   /* sum m |v| (scale for relative momentum error) */
    double rho_abs_max;        /* max_H |rho_n| */
} sce_diag;

/* Create a context for a periodic box of side L with modes max|n_i| <= n_max.
 * shape_kind: sce_shape_kind; shape_width: Gaussian width a or tent half-width
 * (ignored for SCE_SHAPE_DELTA).  Builds the mode and Green-function tables on
 * the current HIP device.  Defaults: eps0 = 1, SCE_PREC_FP64, SCE_SCHEME_KDK,
 * a stream owned by the context.
 * Errors: SCE_EINVAL if L <= 0 or non-finite, n_max < 1 or n_max > 64,
 * shape_width < 0 or non-finite, unknown shape_kind, out == NULL. */
sce_status sce_create(double L, int32_t n_max, int32_t shape_kind, double shape_width,
                      sce_ctx *out);

/* Two-dimensional context: line charges in the periodic square [0, L)^2 of
 * area A = L^2, the setting of the paper's own test problems (Section 6, the
 * two-body problem; Section 7, the thermal plasma).  Modes n in Z^2 with
 * max|n_i| <= n_max, n != 0; half plane H2 = { n_x > 0 } u { n_x = 0, n_y > 0 },
 * |H2| = ((2 n_max + 1)^2 - 1) / 2, canonical order n_x = 0..n_max, then
 * n_y = -n_max..n_max.  The deposit, force, energies and steps are the model
 * above with two components and A in place of V: psi_n = S(k_n) rho_n /
 * (eps0 |k_n|^2 A), W = (1/(eps0 A)) sum_{H2} |rho|^2/|k|^2; S(k) takes the
 * two-component k (tent: sinc^2(k_x a/2) sinc^2(k_y a/2)).  In a 2-D context
 * every array of particle vectors (x, v, F and the checkpoint's contents as
 * seen through sce_set_particles/sce_get_particles) is [2][N], sce_modes
 * writes 2 ints per mode, and sce_diag.momentum[2] is 0.  Every precision
 * and scheme is available.  Arguments and errors as for sce_create. */
sce_status sce_create_2d(double L, int32_t n_max, int32_t shape_kind, double shape_width,
                         sce_ctx *out);

/* Spatial dimension of the context (3, or 2 for sce_create_2d). */
sce_status sce_dimension(sce_ctx ctx, int32_t *dim);

/* Finite-width field shapes (Section 3, the potential's expansion and the
 * k-squared matrix; Section 4, the discrete Euler-Lagrange equations), the
 * variant the paper describes and then sets aside.  The potential is
 * expanded over modes s in the full cube {-n_max..n_max}^D, s = 0 included,
 * k_s = dk s, dk = 2 pi / L, each spread over k-space by a tent
 * Psi(k - k_s) = prod_d max(0, 1 - |k_d - k_s,d| / dk); neighbouring tents
 * overlap, so the potential's transform is piecewise linear.  The field
 * lives on all of R^D: there is no periodic box and positions are never
 * wrapped.  Particles are points (Lambda = delta), which gives the
 * particle-mode integral the closed form f_s(x) = e^{i k_s.x} E(x),
 * E(x) = prod_d (2 pi)^(-1/2) dk sinc^2(dk x_d / 2).  Then
 *   deposit  rho_s = sum_j q_j E(x_j) e^{-i k_s.x_j}, the conjugate of the
 *            paper's right-hand side sum_j q_j f_s(x_j);
 *   solve    eps0 sum_s' K_{s s'} phi_s' = conj(rho_s),
 *            K_{s s'} = int |k|^2 Psi(k - k_s) Psi(-k - k_s') dk, solved exactly
 *            (eps0 = 1/(4 pi) gives the Gaussian-unit factor 4 pi);
 *   force    F_j = -q_j sum_s phi_s grad f_s(x_j); Phi_j = sum_s phi_s f_s(x_j);
 *   energy   W = (eps0/2) phi^T K phi = (1/2) sum_j q_j Phi_j.
 * Translations are not a symmetry, so momentum is not conserved (a lone
 * particle away from the origin feels a force); the steps are those of the
 * periodic model without the wrap.  dim: 3, or 2 (line charges with the
 * conventions of sce_create_2d: arrays [2][N], 2 ints per mode).  The stored
 * modes are the origin followed by H in canonical order, |H| + 1 of them:
 * sce_mode_count, sce_modes, sce_deposit, sce_psi (which returns phi) and the
 * rho_abs of sce_diagnostics use that set.  Every precision and scheme is
 * available.  Errors: SCE_EINVAL if L <= 0 or non-finite, n_max < 1 or
 * n_max > 64, dim not 2 or 3, out == NULL. */
sce_status sce_create_tent(double L, int32_t n_max, int32_t dim, sce_ctx *out);

/* Field shape of the context: SCE_FIELD_DELTA or SCE_FIELD_TENT. */
sce_status sce_field_shape(sce_ctx ctx, int32_t *field);

/* eps0 > 0; precision: sce_precision; scheme: sce_scheme; hip_stream: a
 * hipStream_t on the context's device, or NULL for the context's own stream.
 * Invalidates cached fields.  SCE_EINVAL on bad values. */
sce_status sce_set_options(sce_ctx ctx, double eps0, int32_t precision, int32_t scheme,
                           void *hip_stream);

/* Copy N particles into the context.  x, v: [3][N]; q, m: [N] (m > 0).
 * Positions outside [0, L) are accepted and wrapped (kept as given in a
 * tent-field context).  Resets the step counter
 * and the cached force.  SCE_EINVAL if N < 1, N >= 2^32 or a pointer is
 * NULL (nothing is changed), or if any x, v or q is not finite or any m is
 * not finite and > 0 (checked on the device after the copy; the context then
 * holds no particles); SCE_ENOMEM if the particle arrays do not fit in device
 * memory (the context then holds no particles). */
sce_status sce_set_particles(sce_ctx ctx, int64_t N, const double *x, const double *v,
                             const double *q, const double *m, int32_t on_device);

/* Copy positions and velocities out ([3][N] each; either may be NULL). */
sce_status sce_get_particles(sce_ctx ctx, double *x, double *v, int32_t on_device);

/* Number of stored half-space modes |H| (|H| + 1 with tent fields). */
sce_status sce_mode_count(sce_ctx ctx, int64_t *n_half);

/* The stored modes in canonical order: nxyz[3*i + d] = n_d of mode i (2 ints
 * per mode in a 2-D context).  Host memory. */
sce_status sce_modes(sce_ctx ctx, int32_t *nxyz);

/* Deposit at the current positions: rho [2 |H|] interleaved (re, im), canonical
 * mode order, FP64.  rho may be NULL (result kept on the device only). */
sce_status sce_deposit(sce_ctx ctx, double *rho, int32_t on_device);

/* psi_n = S(k_n) rho_n / (eps0 |k_n|^2 V) from the last deposit, [2 |H|] (re, im). */
sce_status sce_psi(sce_ctx ctx, double *psi, int32_t on_device);

/* Force at the current positions (deposit, solve, force): F [3][N] FP64.
 * Velocities are not changed.  F may be NULL. */
sce_status sce_force(sce_ctx ctx, double *F, int32_t on_device);

/* sce_force without device allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc): the same pass (deposit, solve, force at the current
 * positions) and the same F, but the pass's scratch buffers (phase tables,
 * per-split deposit partials or particle records, the force's line-group
 * partials) live in one static 64 MiB device array per GPU instead of the
 * context's buffers, which sce_force allocates on first use.  The context's
 * own buffers (particles, modes, fields) are allocated by sce_create,
 * sce_set_options and sce_set_particles, as for every call.  Every call of
 * this function on a GPU uses that GPU's one array, which keeps the last
 * call's contents; calls that overlap in time on one GPU (other threads, or
 * other contexts' streams) race and must be ordered by the caller.  Kernel
 * timing (sce_timing_enable) does not record this call.  Errors as
 * sce_force; SCE_EINVAL if the pass needs more than 64 MiB of scratch (for
 * example 65,536 particles at n_max = 16 need about 27 MB with
 * SCE_PREC_SPLIT_F16; 262,144 particles at n_max = 16 need more than 64 MiB
 * with SCE_PREC_FP64). */
sce_status sce_force_noalloc(sce_ctx ctx, double *F, int32_t on_device);

/* Advance n_steps >= 0 steps of size dt (finite) with the configured scheme.
 * Small FP64 systems run as one kernel per block of steps (sce_set_small_step).
 * Otherwise, with n_steps >= 2 G (G = steps per graph, see sce_set_step_graph) and
 * timing off, the first step runs directly, then blocks of G steps replay a
 * HIP graph of their launches (captured again whenever dt, the scheme, the
 * particles or the options change), then the rest run directly.  Results are
 * identical to launching every step directly. */
sce_status sce_step(sce_ctx ctx, double dt, int64_t n_steps);

/* Small systems: sce_step runs an FP64, delta-field context with N <= 256,
 * |H| <= 3072, N (n_max + 1) <= 1024 and N |H| <= max_pairs as one
 * single-workgroup kernel per block of up to 4096 steps (the phase tables,
 * deposit, solve, force, kicks and drift of every step as stages of one
 * launch, the state kept on chip), unless kernel timing is enabled.  Such a
 * step is otherwise bound by the latency of its five kernels.  Results agree
 * with the multi-kernel step to rounding (not bit for bit).  max_pairs in
 * 0..2^24 (0: never; default 65536).  SCE_EINVAL outside the range. */
sce_status sce_set_small_step(sce_ctx ctx, int64_t max_pairs);

/* Steps per captured graph for sce_step, 0..4096 (0: launch every step
 * directly; default 8).  Replaying a graph removes the host's per-launch
 * cost and the gaps between kernels.  SCE_EINVAL outside the range. */
sce_status sce_set_step_graph(sce_ctx ctx, int32_t steps_per_graph);

/* Diagnostics at the current state; rho_abs (|H| doubles, host) may be NULL.
 * Runs a deposit if the fields are not current.  Returns SCE_EUNSTABLE (with
 * *out filled) if the energy is not finite. */
sce_status sce_diagnostics(sce_ctx ctx, sce_diag *out, double *rho_abs);

/* Checkpoint: with buf == NULL, *bytes receives the size needed.  Otherwise
 * buf (host, *bytes long) receives positions, velocities, charges, masses,
 * the step counter and the cached force.  SCE_EINVAL if *bytes is too small. */
sce_status sce_get_state(sce_ctx ctx, void *buf, size_t *bytes);

/* Restore a checkpoint written by sce_get_state for the same L, n_max,
 * dimension and field shape (SCE_EINVAL otherwise).  The saved force is
 * reused only if the particle shape, its width, eps0 and the precision also
 * match; otherwise the next step recomputes it at the restored positions. */
sce_status sce_set_state(sce_ctx ctx, const void *buf, size_t bytes);

/* Wait for all work on the context's stream. */
sce_status sce_sync(sce_ctx ctx);

/* Kernel timing with HIP events recorded on the context's stream.  While
 * enabled, every launch of the deposit kernel (the particle x mode sum of the
 * deposit) and of the force kernel (the particle x mode sum of the force, with
 * its fused kick) is bracketed by a pair of events.  Enabling or disabling
 * synchronises the stream and clears the totals. */
sce_status sce_timing_enable(sce_ctx ctx, int32_t enable);

/* Synchronise, then return the summed event time (ms) and launch count of
 * each kernel since timing was enabled.  Any output pointer may be NULL. */
sce_status sce_timing_read(sce_ctx ctx, double *deposit_ms, int64_t *deposit_launches,
                           double *force_ms, int64_t *force_launches);

/* Release the context and its device memory.  NULL is ignored. */
void sce_destroy(sce_ctx ctx);

const char *sce_status_string(sce_status s);

/* Last error message of this context ("" if none). */
const char *sce_last_error(sce_ctx ctx);

/* ------------------------------------------------------------------ serving
 * Batched serving of many independent small simulations (each one the model
 * above, with its own L, n_max, shape and particles) on one GPU.  Their state
 * stays resident in one device arena; each sce_server_tick advances every
 * resident request by one leapfrog pass with one launch per phase (deposit,
 * solve, force with kick and drift, diagnostics) for all of them together.
 * A request of S steps takes S + 1 passes: the kick-drift-kick step of
 * Section 4 with the kicks of consecutive steps merged (h/2 on the first and
 * last pass, h in between), which gives the same states as S calls of the
 * single-simulation step.  Requests are admitted first-in first-out while
 * their device footprint fits the arena and a slot is free.
 * A server is not thread-safe; its calls synchronise its stream. */
typedef struct sce_server_s *sce_server;

typedef struct {
    size_t hbm_budget_bytes;  /* device arena for resident requests; 0 = 4 GiB */
    int32_t precision;        /* SCE_PREC_FP32 or SCE_PREC_FP64 */
    int32_t max_active;       /* resident requests at most; 0 = 4096 */
    int32_t no_graph;         /* 0: each tick replays a HIP graph of its launches, captured again
                                 whenever the resident set changes; 1: launch directly */
    void *hip_stream;         /* hipStream_t, or NULL for a server-owned stream */
} sce_server_opts;

typedef struct {
    double L, a, eps0, dt;    /* box side (> 0), shape width (>= 0), eps0 (> 0), step (finite) */
    int32_t n_max;            /* 1 .. 16 */
    int32_t shape_kind;       /* sce_shape_kind */
    int64_t N;                /* particles, >= 1 */
    int64_t n_steps;          /* >= 0 */
    const double *x, *v;      /* host [3][N] ([2][N] when dim = 2); positions outside [0, L) are
                                 wrapped by the first drift */
    const double *q, *m;      /* host [N]; m > 0 */
    int32_t dim;              /* 3 (or 0): the periodic cube; 2: line charges in the periodic
                                 square with the conventions of sce_create_2d (x, v and the
                                 result's x, v, F are [2][N], the area L^2 replaces V) */
} sce_request;

typedef struct {
    int64_t ticks;            /* ticks that advanced at least one request */
    int64_t request_steps;    /* passes completed, summed over requests */
    int64_t requests_done;
    int64_t active, queued;   /* now */
    double busy_s;            /* wall time inside those ticks */
    double pairs;             /* sum over ticks of sum over resident requests of N |H| */
    double p50_step_s, p99_step_s, max_step_s;  /* per request-pass latency: the wall time of the
                                                   tick that carried it (admission, launches,
                                                   retirement included) */
    double p50_wait_s, p99_wait_s;              /* admission wait: submit to the start of the
                                                   first tick that carried the request */
    double hbm_used_bytes, hbm_peak_bytes;      /* arena bytes held by resident requests */
    double gpu_p50_step_s, gpu_p99_step_s;      /* per request-pass device time of the tick's
                                                   kernels alone (HIP events around its
                                                   launches), weighted like p50/p99_step_s:
                                                   the rest of a step's latency is the host's */
} sce_server_report;

/* Create a server on the current HIP device.  opts may be NULL (defaults).
 * Errors: SCE_EINVAL (out == NULL, max_active < 0), SCE_ENOTSUP (precision
 * other than FP32 or FP64), SCE_ENOMEM (arena allocation failed). */
sce_status sce_server_create(const sce_server_opts *opts, sce_server *out);

/* Queue a request; its arrays are copied before returning.  *id (> 0) names it.
 * Errors: SCE_EINVAL for invalid fields, or if its footprint exceeds the whole
 * arena (it could never be admitted). */
sce_status sce_server_submit(sce_server s, const sce_request *req, uint64_t *id);

/* Admit what fits, then run one pass of every resident request and retire the
 * finished ones (their results move to host memory).  n_active and n_queued
 * (may be NULL) receive the counts after the tick. */
sce_status sce_server_tick(sce_server s, int32_t *n_active, int32_t *n_queued);

/* Ids of requests finished since the last poll, oldest first, at most max. */
sce_status sce_server_poll(sce_server s, uint64_t *done_ids, int32_t max, int32_t *n_done);

/* Result of a finished request, then forgotten: x, v, F host [3][N] ([2][N]
 * for a two-dimensional request) at the end (F at the final positions), diagnostics at the start (first) and the
 * end (last).  Any output may be NULL.  SCE_EINVAL if id is not finished or
 * was already fetched. */
sce_status sce_server_result(sce_server s, uint64_t id, double *x, double *v, double *F,
                             sce_diag *first, sce_diag *last);

sce_status sce_server_stats(sce_server s, sce_server_report *out);

/* Last error message of this server ("" if none). */
const char *sce_server_last_error(sce_server s);

/* Release the server, its arena and all unfetched results.  NULL is ignored. */
void sce_server_destroy(sce_server s);

#ifdef __cplusplus
}
#endif

#endif /* SCE_H */
