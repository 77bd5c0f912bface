/*
 * pss.h -- C interface of the MI355X pseudo-spectral stochastic-PDE stepper.
 *
 * The library advances real fields phi_f on a periodic 1D, 2D or 3D lattice with
 * the semi-implicit Euler-Maruyama scheme of cuPSS (arXiv 2405.02410,
 * eq:timeupdate and the six-step list that follows it):
 *
 *   phi_f(t+dt) = ( phi_f + dt * sum_t M_t(q) N_t + sigma_f(q) xi_f ) / (1 - dt L_f(q))
 *
 * where L_f is the sum of the field's implicit operators, each explicit term t
 * contributes M_t(q) times the Fourier transform of a product of de-aliased
 * fields evaluated in real space (eq:basereal, eq:nonlin_general), and the
 * noise has Fourier variance 2 D_f(q) (eq:noise_eq, Sec. "Adding noise").
 *
 * The calls follow the paper's statement of a problem (Sec. "Writing
 * models"): create a system from sizes, spacings and dt; declare fields; add
 * implicit and explicit terms; add noise; set initial conditions; evolve.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every function returns a pss_status: PSS_OK (0) or a negative code.  No
 *   exception or abort crosses the interface.  pss_last_error() returns a
 *   thread-local message describing the most recent failure on the calling
 *   thread.
 * - Sizes are given as n[3] = {Nx, Ny, Nz} and dx[3] = {dx, dy, dz}; a 2D
 *   lattice ignores n[2] and dx[2], a 1D lattice n[1], n[2], dx[1], dx[2].
 *   Every N_i must be a power of two in [8, 4096]; other sizes return
 *   PSS_E_UNSUPPORTED.
 * - Real-space arrays are float32, x fastest: index (z*Ny + y)*Nx + x.
 * - Fourier convention: forward transform unnormalised, inverse with 1/N.
 *   Mode indices are signed integers in FFT order with the Nyquist index read
 *   as -N_i/2; q_i = 2 pi k_i / (N_i dx_i).
 * - Terms are written on the right-hand side of d/dt phi.  The paper's
 *   equation string "dt phi + lhs = rhs" therefore maps to implicit operators
 *   equal to minus the lhs prefactor (Sec. "Writing models").
 * - The context owns every device buffer it allocates.  Host arrays passed in
 *   are copied before the call returns; device pointers passed with
 *   on_device = 1 must stay valid until the call returns.
 * - pss_step is asynchronous on the context's stream; device faults surface
 *   as PSS_E_HIP at the next synchronising call (pss_sync, downloads, saves).
 * - Structural calls (declare, term_add, noise_set, dealias_set) are only
 *   accepted before the device plan is built (first upload, init or step);
 *   afterwards they return PSS_E_STATE.  Coefficients can still be changed
 *   with pss_term_set_coef, and pss_noise_set with the monomials unchanged.
 * - A context is not thread-safe: one thread at a time.
 */
#ifndef PSS_H
#define PSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pss_ctx pss_ctx;
typedef struct pss_batch pss_batch;
typedef struct pss_tape pss_tape;
typedef int32_t pss_status;

#define PSS_OK 0
#define PSS_E_INVAL (-1)       /* bad argument (null pointer, index, size) */
#define PSS_E_UNSUPPORTED (-2) /* valid request outside what is implemented */
#define PSS_E_NOMEM (-3)       /* device allocation failed */
#define PSS_E_HIP (-4)         /* a HIP runtime call or kernel failed */
#define PSS_E_STATE (-5)       /* call not allowed in the current state */
#define PSS_E_UNSTABLE (-6)    /* 1 - dt*L(q) has real part <= 0 on some mode */
#define PSS_E_NONFINITE (-7)   /* a NaN or infinity appeared in the state (reported by pss_sync) */

/* De-aliasing (Sec. "De-aliasing").  A factor entering nonlinear terms of
 * highest order n has its modes beyond a fraction f of the Nyquist index
 * zeroed before the real-space product: TWO_THIRDS uses f = 2/3 for every
 * factor, PAPER_ORDER uses f = 2/(n+1) (the paper's |q| > 2 pi/((n+1) dx)
 * rule), NONE keeps every mode.  RADIAL keeps sum_i (k_i/(N_i/2))^2 < f^2,
 * PER_AXIS keeps |k_i|/(N_i/2) < f on every axis.  Modes on the cutoff are
 * zeroed. */
#define PSS_DEALIAS_TWO_THIRDS 0
#define PSS_DEALIAS_PAPER_ORDER 1
#define PSS_DEALIAS_NONE 2
#define PSS_SHAPE_RADIAL 0
#define PSS_SHAPE_PER_AXIS 1

/* One operator monomial (Sec. "Reserved keywords"):
 *   coef * (q^2)^q2_pow * |q|^(-invq_pow) * (i qx)^iq_pow[0] (i qy)^iq_pow[1] (i qz)^iq_pow[2]
 * q^2 is -laplacian, i q_i is d/dx_i (zero on the Nyquist plane of axis i),
 * 1/|q| is zero at q = 0.  An operator is a sum of monomials.  All powers
 * must lie in [0, 8]. */
typedef struct {
    double coef;
    int32_t q2_pow;
    int32_t invq_pow;
    int32_t iq_pow[3];
} pss_qmono;

/* ---- lattice ----------------------------------------------------------- */

/* Create a lattice context (Sec. "Writing models", the system constructor).
 * ndim: 1, 2 or 3.  n, dx: see conventions.  dt > 0.  Touches no device: the
 * device plan is built on the first upload, init or step.  A 1D lattice (the
 * line of the examples in Sec. "Callback functions" and "De-aliasing") is
 * stepped by one block that holds the whole line; its state is the full
 * complex spectrum of the line (pss_state_size), and it takes part in neither
 * batches nor the adjoint (PSS_E_UNSUPPORTED there).  A size may also be an
 * even 2^a 3^b 5^c (Sec. "Benchmarking": sizes other than powers of two are
 * allowed, at a lower speed).  Such lattices run on a generic path: the
 * state of a field is its full complex spectrum (mode (kx, ky, kz) at
 * (kz Ny + ky) Nx + kx; pss_state_size and pss_field_state_bytes count it),
 * each line is transformed in LDS, which bounds the line length times the
 * field and factor counts (PSS_E_UNSUPPORTED when the plan is built, with the
 * bytes it would need), and a 2D or 3D one takes part in neither batches,
 * the adjoint nor pss_time_kernel (PSS_E_UNSUPPORTED).
 * Errors: PSS_E_INVAL (null out, dt <= 0, dx <= 0), PSS_E_UNSUPPORTED (ndim
 * not 1, 2 or 3, a size outside [8, 4096] or not an even 2^a 3^b 5^c). */
pss_status pss_lattice_create(pss_ctx **out, int32_t ndim, const int64_t n[3],
                              const double dx[3], double dt);

/* Release the context and every buffer it owns.  NULL is accepted. */
pss_status pss_lattice_destroy(pss_ctx *ctx);

/* ---- model ------------------------------------------------------------- */

/* Declare a field (Sec. "Writing models", createField).  dynamic = 1 for a
 * field with its own time derivative (at most 4); dynamic = 0 for an
 * intermediate field (at most 4), defined by an equation without a time
 * derivative, "psi + lhs = rhs" in the paper's notation: its implicit terms
 * (operators on psi itself, written on the right-hand side like those of a
 * dynamic field, so L_psi is minus the lhs prefactor) and its explicit terms
 * give  psi_hat = sum_t M_t phi_t_hat / (1 - L_psi(q)).  The paper's example
 * psi + psi q^2 = -q^2 phi is the implicit term -q^2 psi and the explicit
 * term -q^2 phi.  Each explicit term of an intermediate field must be one
 * dynamic field to the first power (PSS_E_UNSUPPORTED otherwise, also for an
 * intermediate source).  Intermediate fields enter the terms of dynamic fields
 * as factors of products (de-aliased like any factor) or as sources of linear
 * terms; they are evaluated from the step-n state, as step 1 of the per-step
 * list after eq:timeupdate.  Names must be unique over both kinds, 1..63
 * characters.  *field_id receives the declaration index (0, 1, ...), which
 * every other call takes and which keys the field's random numbers. */
pss_status pss_field_declare(pss_ctx *ctx, const char *name, int32_t dynamic,
                             int32_t *field_id);

/* Add a term  op(q) * prod_j field_j^power_j  to d/dt of target_field
 * (eq:basereal; the operator acts on the whole product, Sec. "Writing
 * models"), or to the equation of an intermediate target (see
 * pss_field_declare).  implicit = 1 requires exactly one factor, the target field to
 * the power 1 (implicit terms must be linear in their field); its operator is
 * added to L(q).  Explicit terms: 1 to 4 factors with powers 1..8; a single
 * factor of power 1 is applied directly in Fourier space, any other term is
 * formed in real space from de-aliased factors.  At most 8 monomials per
 * operator, 32 terms in total.  When the plan is built, the real-space terms
 * become product channels: terms of one target with the same single-monomial
 * operator shape share a channel, and a channel whose products equal
 * another's up to a common factor for a different target is folded into it
 * (one transform feeds both updates).  A model may use at most 8 channels and
 * 8 distinct factor fields in its products (PSS_E_UNSUPPORTED otherwise,
 * reported when the plan is built).  *term_id (may be NULL) receives the
 * index. */
pss_status pss_term_add(pss_ctx *ctx, int32_t target_field, int32_t implicit,
                        const pss_qmono *op, int32_t n_mono,
                        const int32_t *factor_fields, const int32_t *factor_powers,
                        int32_t n_factors, int32_t *term_id);

/* Read back term `term_id` as added: its target, implicit flag, operator
 * (op receives *n_mono monomials; pass room for 8) and factors (room for 4);
 * every pointer may be NULL.  pss_term_count gives the number of terms. */
pss_status pss_term_info(pss_ctx *ctx, int32_t term_id, int32_t *target, int32_t *implicit, pss_qmono *op,
                         int32_t *n_mono, int32_t *factor_fields, int32_t *factor_powers, int32_t *n_factors);
pss_status pss_term_count(pss_ctx *ctx, int32_t *count);

/* Change the coefficient of monomial `mono` of term `term_id`.  Allowed at
 * any time; takes effect at the next step (stream-ordered).  Re-checks
 * stability: PSS_E_UNSTABLE leaves the old value in place. */
pss_status pss_term_set_coef(pss_ctx *ctx, int32_t term_id, int32_t mono, double coef);

/* Add noise to a field (Sec. "Adding noise"): D(q) is a sum of monomials in
 * q^2 and 1/|q| only (no i q_i), real and >= 0 on every mode (checked when the
 * plan is built; PSS_E_INVAL otherwise).  The Fourier noise amplitude is
 * sigma(q) = sqrt(2 D(q) dt / dV) on unit white noise.  After the plan is
 * built, a call that repeats the field's monomials with new coefficients is a
 * coefficient change (takes effect at the next step); any other call then
 * returns PSS_E_STATE. */
pss_status pss_noise_set(pss_ctx *ctx, int32_t field, const pss_qmono *D_of_q,
                         int32_t n_mono);

/* ---- equation front end ------------------------------------------------ */

/* Named parameter for equation strings (Sec. "Writing models",
 * addParameter): a finite value, substituted when an equation or a noise
 * prefactor that names it is added (later changes do not reach terms already
 * added; pss_term_set_coef does).  Names follow the field-name rules. */
pss_status pss_param_set(pss_ctx *ctx, const char *name, double value);
pss_status pss_param_get(pss_ctx *ctx, const char *name, double *value);

/* The declaration index of the field called `name` and whether it is dynamic
 * (either pointer may be NULL); PSS_E_INVAL if there is none. */
pss_status pss_field_find(pss_ctx *ctx, const char *name, int32_t *field_id, int32_t *dynamic);

/* Add the terms of one equation written as in Sec. "Writing models":
 *   "dt phi + (a*q^2 + k*q^4)*phi = -b*q^2*phi^3"   (dynamic field phi)
 *   "psi + psi*q^2 = -q^2*phi"                        (intermediate field psi)
 * "dt NAME" opens the equation of a dynamic field, a bare NAME that of an
 * intermediate field (it must have been declared so).  After the field, the
 * left-hand side may hold terms linear in it, each "operator * field"
 * (implicit terms; moved to the right-hand side with the opposite sign); the
 * right-hand side is a sum of products of numbers, parameters, fields with
 * integer powers, the keywords q^2n ((-laplacian)^n), iqx, iqy, iqz (the
 * derivatives) and "/q" (1/|q|), and parenthesised sums, each factor joined
 * by '*' (Sec. "Reserved keywords").  Monomials with equal field factors are
 * gathered into one term (up to 8 monomials a term).  *first_term and
 * *n_terms (either may be NULL) receive the id of the first term added and
 * the number added (ids are consecutive).  Errors: PSS_E_INVAL (syntax, an
 * unknown name, a non-linear left-hand side, 'dt' on an intermediate field
 * or its absence on a dynamic one; the message gives the position),
 * PSS_E_UNSUPPORTED (a term without fields), and those of pss_term_add.  A
 * failure in pss_term_add can leave earlier terms of the equation added. */
pss_status pss_equation_add(pss_ctx *ctx, const char *equation, int32_t *first_term, int32_t *n_terms);

/* Noise of `field` from a prefactor string, e.g. "D*q^2" (Sec. "Adding
 * noise", addNoise): numbers, parameters, q^2n and /q only; then as
 * pss_noise_set. */
pss_status pss_noise_expr(pss_ctx *ctx, int32_t field, const char *expr);

/* Boundary frame (Sec. "Callback functions": a field held at fixed values on
 * a band of sites, the buffer zone that imposes a boundary condition on a
 * periodic lattice).  After the update of every step, the real space of
 * dynamic field `field` (the real part of its inverse transform) takes
 * values[i] at linear site sites[i] = (z*Ny + y)*Nx + x, i < n, and the
 * field is transformed back; the next step starts from that state.  n = 0
 * removes the field's frame.  Arrays are host memory, copied.  In 1D the
 * frame is applied inside the step launch; in 2D and 3D it adds a pass
 * through real space and a rebuild of the channel arrays after every step.
 * Errors: PSS_E_INVAL (an intermediate field, a site off the lattice, a
 * non-finite value), PSS_E_STATE (while a batch or an adjoint tape holds the
 * lattice).  Lattices with frames take part in neither batches nor the
 * adjoint (PSS_E_UNSUPPORTED there). */
pss_status pss_frame_set(pss_ctx *ctx, int32_t field, const int64_t *sites, const float *values, int64_t n);

/* 64-bit seed of the Philox4x32-10 noise (Salmon et al. SC'11).  The noise of
 * mode k of field f at step n is keyed by counter (c(k), n, f, 0) with key
 * (low, high) words of the seed, where c(k) = min(L(k), L(-k)) and L is the
 * linear mode index (z*Ny + y)*Nx + x of the full spectrum.  Default 0. */
pss_status pss_seed_set(pss_ctx *ctx, uint64_t seed);

/* De-aliasing rule and shape (defaults TWO_THIRDS, RADIAL). */
pss_status pss_dealias_set(pss_ctx *ctx, int32_t rule, int32_t shape);

/* Run on this hipStream_t (NULL selects the context's own stream).  The
 * caller keeps the stream alive while the context uses it.  The legacy null
 * stream cannot host graph capture; pass a created stream.  PSS_E_STATE while
 * a batch or an adjoint tape holds the context (they order their work on the
 * streams the members had when they were made). */
pss_status pss_stream_set(pss_ctx *ctx, void *hip_stream);

/* Launch-geometry override, before the plan is built (PSS_E_STATE after).
 * Keys: "tc" (packed columns per tile; also the array layout), "to" (3D:
 * y lines per update block), "tz" (3D: z lines per y-pass block), "rb" (rows
 * per x-kernel block), "pu", "px", "py" (points per thread of the update,
 * x and y kernels: 4, 8 or 16).  On a lattice with a size that is not a
 * power of two (2D, 3D) only "tc" (lines per column-kernel block) and "py"
 * (3D: lines per y-pass block) apply, each a divisor of Nx up to 64 whose
 * block fits the LDS.  value <= 0 restores the default.  Invalid
 * combinations are reported as PSS_E_UNSUPPORTED when the plan is built. */
pss_status pss_tuning_set(pss_ctx *ctx, const char *key, int64_t value);

/* The geometry value in use for a key (builds the plan if needed). */
pss_status pss_tuning_get(pss_ctx *ctx, const char *key, int64_t *value);

/* Check the model without touching the device: implicit terms, noise
 * operators, stability Re(1 - dt L(q)) > 0 on every mode of every dynamic
 * field, and |1 - L_psi(q)| > 1e-6 max(1, |L_psi(q)|) on every mode of every
 * intermediate field (PSS_E_UNSTABLE otherwise). */
pss_status pss_validate(pss_ctx *ctx);

/* ---- state ------------------------------------------------------------- */

/* Set field from a real-space float32 array (host, or device if on_device).
 * Synchronous: returns after the forward transform has completed.  Dynamic
 * fields only (PSS_E_INVAL for an intermediate field); the same holds for
 * pss_field_init_uniform, pss_spectrum_download, pss_mass and the
 * structure-factor calls. */
pss_status pss_field_upload(pss_ctx *ctx, int32_t field, const float *real_xyz,
                            int32_t on_device);

/* Set field to float32(lo + (hi - lo) u) at every site, u the first uniform of
 * Philox counter (site, 0, field, 1) with the context seed; u is an odd
 * multiple of 2^-24 in (0, 1).  Synchronous. */
pss_status pss_field_init_uniform(pss_ctx *ctx, int32_t field, double lo, double hi);

/* Write the real-space field (inverse transform of the full state, no
 * de-aliasing) to a float32 array.  An intermediate field is computed on the
 * device from the current state of the dynamic fields.  Synchronous. */
pss_status pss_field_download(pss_ctx *ctx, int32_t field, float *real_xyz,
                              int32_t on_device);

/* Write the Fourier state of a field as the half spectrum: complex float32
 * pairs (re, im) of modes kx = 0..Nx/2 for every (z, y), index
 * ((z*Ny + y)*(Nx/2+1) + kx).  Synchronous. */
pss_status pss_spectrum_download(pss_ctx *ctx, int32_t field, float *half_spectrum,
                                 int32_t on_device);

/* Advance nsteps time steps (eq:timeupdate).  nsteps = 0 is a no-op.
 * Asynchronous on the context stream; replays captured HIP graphs of the
 * step sequence.
 * Debug mode: a lattice created while the environment variable
 * PSS_DEBUG_SYNC is set (and not "0") enqueues the same kernels one step at
 * a time without graphs, synchronises the stream after every kernel, and
 * returns PSS_E_HIP or PSS_E_NONFINITE from pss_step itself, naming the
 * kernel and the step; its workspaces start filled with NaN so that a read
 * before a write would reach the state.  Results are bitwise those of the
 * graph path.  After such an error the state is undefined and the step
 * index counts the completed steps.  Batches and tapes are not affected. */
pss_status pss_step(pss_ctx *ctx, int64_t nsteps);

/* Build the plan (if needed) and capture and instantiate the HIP graphs that
 * pss_step(ctx, nsteps) replays (chunks of up to 50 steps and the remainder),
 * without running them.  The state is unchanged.  For callers that time or
 * capture pss_step and want no graph construction inside that region.
 * Errors: PSS_E_INVAL (nsteps < 0), plan errors as for pss_step. */
pss_status pss_step_prepare(pss_ctx *ctx, int64_t nsteps);

/* Number of steps taken since the plan was built (the noise step index). */
pss_status pss_step_index(pss_ctx *ctx, int64_t *out);

/* Wait for the context stream; reports asynchronous device failures.  The
 * update kernel raises a device flag when a new state value is NaN or
 * infinite (a blown-up run); pss_sync then returns PSS_E_NONFINITE once, with
 * the mask of the affected fields in the message, and clears the flag.
 * Uploads, uniform initialisation and state loads also clear it. */
pss_status pss_sync(pss_ctx *ctx);

/* Let caller-owned device memory (for example a torch tensor) hold the
 * Fourier state of dynamic field `field` instead of memory the library
 * allocates.  device_ptr: device memory on the context's device, 8-byte
 * aligned, at least pss_field_state_bytes(field) bytes (`bytes` is the size
 * the caller has); the caller keeps it alive until the lattice is destroyed,
 * and the library never frees it.  Call before the plan is built (the first
 * call that needs the device): PSS_E_STATE afterwards; PSS_E_INVAL for a null,
 * misaligned or short buffer or an intermediate field, and, when the plan is
 * built, for memory that is not device memory.  Building the plan clears it to
 * zero, as it does the library's own.  Layout: the library's packed spectral
 * layout of the field, byte for byte the field's block of pss_state_save.  The
 * library reads and writes it on the context's stream; a caller that writes
 * it directly must then call pss_state_changed. */
pss_status pss_field_bind(pss_ctx *ctx, int32_t field, void *device_ptr, size_t bytes);

/* Bytes of one dynamic field's Fourier state (8 bytes per stored complex
 * mode: (Nx/2) Ny Nz in 2D and 3D, Nx in 1D, Nx Ny Nz for a lattice of
 * mixed-radix sizes). */
pss_status pss_field_state_bytes(pss_ctx *ctx, int32_t field, size_t *bytes);

/* Tell the library that the state changed outside its calls (memory bound
 * with pss_field_bind written by the caller): the next step rebuilds its
 * real-space products from the state. */
pss_status pss_state_changed(pss_ctx *ctx);

/* Bytes needed by pss_state_save. */
pss_status pss_state_size(pss_ctx *ctx, size_t *bytes);

/* Save / restore every field's Fourier state and the step index into a host
 * buffer of pss_state_size bytes.  A restored run replays exactly, because
 * the noise is keyed by (seed, step, mode).  Synchronous. */
pss_status pss_state_save(pss_ctx *ctx, void *dst, size_t bytes);
pss_status pss_state_load(pss_ctx *ctx, const void *src, size_t bytes);

/* ---- reductions -------------------------------------------------------- */

/* Mass sum_x phi(x) (= Re phi_hat(0)), in FP64.  Synchronous. */
pss_status pss_mass(pss_ctx *ctx, int32_t field, double *mass);

/* Shell-averaged structure factor S_j = mean over modes with
 * round(|k|) = j of (dV/N)|phi_hat(k)|^2, j = 1 .. n_shells, n_shells =
 * min_i(N_i)/2 - 1 (Sec. "Example", the coarsening observable); counts[j-1]
 * receives the shell population.  The FP64 terms are summed exactly on the
 * device (each rounded once to 2^-62 of its shell's largest term, then added
 * as integers), so the result does not depend on the order of the device's
 * atomics and repeats bit for bit.  A shell with a NaN term is NaN; one with
 * an infinite term and no NaN is +inf.  Synchronous. */
pss_status pss_structure_factor(pss_ctx *ctx, int32_t field, double *S, int64_t *counts,
                                int32_t n_shells);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc: tight serving or monitoring loops, harnesses that forbid it):
 * the result of pss_structure_factor, computed without any device or host
 * allocation.  The shell sums and counts live in a static device array of the
 * library (64 KiB per GPU, held until the process ends) instead of buffers
 * allocated on first use; n_shells above 2047 is PSS_E_UNSUPPORTED (every
 * lattice of at most 4096 per axis fits).  The plan must already be built
 * (PSS_E_STATE otherwise: building it allocates).  Writes S and counts as
 * pss_structure_factor does; synchronous on the context's stream.  All calls
 * on one GPU share the array: calls that overlap in time on one GPU (other
 * threads, other streams) race and must be serialised by the caller. */
pss_status pss_structure_factor_noalloc(pss_ctx *ctx, int32_t field, double *S, int64_t *counts,
                                        int32_t n_shells);

/* ---- utilities --------------------------------------------------------- */

/* Philox4x32-10 words for counters (c0 + i, c1, c2, c3), i = 0..count-1, with
 * key (k0, k1), written as 4*count uint32 to device memory `out_device` (the
 * same device routine the noise uses).  Synchronous. */
pss_status pss_util_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                           uint32_t k0, uint32_t k1, int64_t count, uint32_t *out_device);

/* Benchmark helper: launch kernel `which` of one step `reps` times back to
 * back on the context stream between two HIP events and return the mean
 * time per launch in milliseconds.  which = 0 is the update kernel (the last
 * axis: y in 2D, z in 3D), 1 the x (real-space product) kernel, 2 and 3 the
 * inverse and forward y passes of 3D lattices.  Destroys the state's
 * physical meaning; for timing only.  *name receives a static kernel name. */
pss_status pss_time_kernel(pss_ctx *ctx, int32_t which, int32_t reps, double *ms_per_launch,
                           const char **name);

/* Pick the launch geometry by timing: before the plan is built, try points
 * per thread and tile widths of the update kernel (pu, tc; 3D: to), then of
 * the x kernel (px, rb), then (3D) of the y passes (py, tz), each on a scratch
 * copy of the model with `reps` back-to-back launches per kernel (HIP
 * events), and keep the fastest as if set by pss_tuning_set.  Keys the
 * caller already set are kept.  The choice is cached for the process per
 * device, lattice shape, term structure and forced keys.  If the environment
 * variable PSS_TUNE_CACHE names a file, a choice missing from the process
 * cache is looked up there first, and a new one is appended to it as the
 * text line "<key> <us per step> <k>=<v> ..." (the last line of a key wins;
 * lines that do not parse are skipped; PSS_E_INVAL if the file cannot be
 * written, with the choice still applied).  *us_per_step (may be NULL)
 * receives the summed kernel time of one step at the choice.  Tiling keys
 * leave results bitwise unchanged; points per thread change the FFT radix
 * and so the FP32 rounding.  PSS_E_STATE after the plan is built. */
pss_status pss_autotune(pss_ctx *ctx, int32_t reps, double *us_per_step);

/* Per-launch algorithmic HBM bytes of kernel `which` (same numbering): the
 * bytes each launch must read and write once at the current plan. */
pss_status pss_kernel_bytes(pss_ctx *ctx, int32_t which, double *bytes);

/* Number of kernels in one step (2 in 2D, 4 in 3D). */
pss_status pss_kernels_per_step(pss_ctx *ctx, int32_t *count);

/* ------------------------------------------------------------------ adjoint
 * Reverse-mode gradient of a structure-factor loss through a 2D Model B
 * trajectory (Sec. "Example": the model; eq:timeupdate: the step that is
 * differentiated; the paper itself has no adjoint).  The lattice must hold
 * exactly the Model B terms: one field, an implicit operator with q^2 and q^4
 * monomials -(a q^2 + k q^4), one explicit term -b q^2 F[phi^3], and either
 * no noise or D(q) = D q^2 (anything else: PSS_E_UNSUPPORTED).
 *
 * From the current state phi_0 at step n0 the call runs nsteps forward steps
 * (noise keyed by steps n0 .. n0+nsteps-1, as pss_step would), keeping a
 * checkpoint of the state every ckpt_every steps.  It evaluates
 *   L = sum_{j=1}^{n_shells} (S_j - S_target[j-1])^2,
 * S_j the shell averages of pss_structure_factor at the final step
 * (n_shells = min(Nx, Ny)/2 - 1), and sweeps back through the steps,
 * recomputing each segment from its checkpoint, with the adjoint recursion
 *   r = g_{n+1} / A,   g_n = r + b m F[3 u_n^2 N F^-1[-dt q^2 r]] / N,
 *   u_n = F^-1[m phi_n],   A = 1 + dt q^2 (a + k q^2),
 * where m is the de-aliasing mask and the noise of each step is regenerated
 * from its Philox counter (it does not depend on the coefficients other than
 * through D).  Outputs: *loss; grad[4] = dL/d(a, b, k, D) (FP64 sums of FP32
 * terms, taken in a fixed order: the same run gives the same bits;
 * dL/dD = 0 when D = 0); grad_phi0 (may be NULL; else Nx*Ny floats,
 * host or device memory per on_device) = dL/dphi_0(x) for the real initial
 * field.  The lattice is left at step n0 + nsteps with the forward final
 * state.  Device workspace: (ceil(nsteps/ckpt_every) + min(ckpt_every,
 * nsteps) + 8) arrays of Nx*Ny*4 bytes, allocated for the call. */
pss_status pss_adjoint_model_b(pss_ctx *ctx, int64_t nsteps, int32_t ckpt_every, const double *S_target,
                               int32_t n_shells, double *loss, double *grad, float *grad_phi0, int32_t on_device);

/* The same gradient in two phases, for callers that need the loss before
 * deciding on the gradient (an autograd forward followed, or not, by a
 * backward).  pss_adjoint_model_b_forward runs the checkpointed forward run
 * and returns the loss and a tape that owns the checkpoints and the reverse
 * workspace (the device memory listed above; PSS_E_NOMEM if it does not fit).
 * pss_adjoint_model_b_backward runs the reverse sweep once and writes grad and
 * grad_phi0 as pss_adjoint_model_b does; it fails with PSS_E_STATE if the
 * lattice's coefficients, seed or state changed after the forward phase, or
 * if the sweep already ran.  pss_tape_destroy frees the tape (NULL accepted).
 * While a tape exists its lattice refuses pss_lattice_destroy,
 * pss_stream_set and a second tape (PSS_E_STATE).  After the forward phase
 * the lattice is at step n0 + nsteps with the forward final state, as after
 * the backward phase. */
pss_status pss_adjoint_model_b_forward(pss_ctx *ctx, int64_t nsteps, int32_t ckpt_every,
                                       const double *S_target, int32_t n_shells, double *loss,
                                       pss_tape **tape);
pss_status pss_adjoint_model_b_backward(pss_tape *tape, double *grad, float *grad_phi0, int32_t on_device);
pss_status pss_tape_destroy(pss_tape *tape);

/* ------------------------------------------------------------------ batches
 * Many independent 2D lattices advanced together.  The paper finds small
 * lattices overhead-bound on the GPU (its benchmarks: the CPU version wins
 * below 128^2, Sec. "Benchmarks"); a batch runs all its lattices in the same
 * launches, so the per-launch cost is paid once and the launches hold enough
 * blocks to fill the chip.
 *
 * Lattices with equal sizes, field count, factor and channel counts and launch
 * geometry form one class.  Every class whose lattices have one field,
 * operators without 1/|q| or i q_i monomials, the default 4 points per thread
 * and lines of 64 to 1024 joins two fused launches per time step: one for the
 * update phase and one for the x phase of all such classes, over a work list
 * of (class, member, tile).  Any other class runs one update launch and one x
 * launch of its own per step, with the lattice picked by blockIdx.y.  Every
 * lattice keeps its own model, coefficients, seed (noise keys), de-aliasing,
 * state and step counter; a batch step gives, bit for bit, the state that
 * pss_step gives on that lattice alone. */

/* Make a batch of n >= 1 distinct 2D lattices (3D lattices: PSS_E_UNSUPPORTED;
 * a lattice listed twice or a null entry: PSS_E_INVAL).  The lattices are
 * planned (as by pss_validate) if they were not.  seeds may be NULL; else
 * seeds[i] is set on lattices[i] as by pss_seed_set.  The batch borrows the
 * lattices: pss_lattice_destroy of a member fails with PSS_E_STATE until every
 * batch holding it is destroyed.  Members stay usable on their own (state I/O,
 * pss_step, pss_term_set_coef, pss_state_load); work on a member's stream is
 * ordered against the batch's steps.  The batch runs on the first lattice's
 * stream.
 *
 * Execution (the small-lattice overhead of Sec. "Benchmarks" is what it
 * removes): members of equal sizes, field/factor/channel counts and launch
 * geometry form a class.  A class of one-field lattices whose products use
 * that field only, with Nx and Ny in {64, 128} and the default 4 points per
 * thread, is LDS-resident: one launch per replayed chunk of steps, one block
 * per member holding its whole lattice on chip (set PSS_BATCH_RESIDENT=0 in
 * the environment before pss_batch_create to turn this off).  The other
 * classes of one-field lattices with lines of 64..1024 share one update
 * launch and one x launch per step over a work list of every class; any
 * remaining class runs its own pair of launches per step.  Every form gives
 * each member bit for bit the state that pss_step gives the lattice alone. */
pss_status pss_batch_create(pss_batch **batch, pss_ctx *const *lattices, int32_t n, const uint64_t *seeds);

/* Wait for the batch's work and free the batch (not its lattices). NULL is a no-op. */
pss_status pss_batch_destroy(pss_batch *batch);

/* Advance every member by nsteps >= 0 steps (asynchronous, like pss_step;
 * captured HIP graphs of up to 50 steps). */
pss_status pss_batch_step(pss_batch *batch, int64_t nsteps);

/* Block until the batch's stream is idle; PSS_E_NONFINITE (as pss_sync) if
 * any member's flag is raised (every member's flag is cleared). */
pss_status pss_batch_sync(pss_batch *batch);

/* Number of size classes; class_of (may be NULL, else n entries) receives the
 * class of each member in creation order. */
pss_status pss_batch_info(pss_batch *batch, int32_t *n_classes, int32_t *class_of);

/* Time `reps` back-to-back launches of one class's update kernel (which = 0)
 * or x kernel (which = 1) with HIP events on the batch stream: *ms per launch;
 * *bytes (may be NULL) the launch's algorithmic HBM bytes (the first member's
 * per-lattice figure times the class size).  cls = -1 times the fused launch
 * of that phase (bytes summed over its classes; PSS_E_INVAL if the batch has
 * none).  cls = -2 times one launch of `reps` steps of every LDS-resident
 * class: *ms per step, *bytes the launch's HBM bytes (state and channel array
 * in and out once) per step; which is then ignored (0 or 1).  Leaves the
 * members' channel arrays stale and moves their states on, so the next step
 * rebuilds the channels; for timing only. */
pss_status pss_batch_time_kernel(pss_batch *batch, int32_t cls, int32_t which, int32_t reps, double *ms,
                                 double *bytes);

/* Kernel launches per time step of the batch outside the LDS-resident
 * classes (2 when every other class is fused), the number of classes in the
 * fused launches, and the number of LDS-resident classes (one launch per
 * replayed chunk of up to 50 steps each); any pointer may be NULL. */
pss_status pss_batch_launches(pss_batch *batch, int32_t *per_step, int32_t *fused_classes,
                              int32_t *resident_classes);

const char *pss_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PSS_H */
