/*
 * teuk.h - C ABI of the MI355X m-mode Teukolsky Lax-Wendroff engine.
 *
 * What it computes (Khanna & McKennon, "Numerical modeling of gravitational
 * wave sources accelerated by OpenCL"):
 *   - Sec. 3.1, Eq. (1): the Teukolsky master equation for spin-weight-s
 *     perturbations of a Kerr black hole (mass M, spin a).
 *   - Sec. 3.2: tortoise coordinate r*, azimuth phi~, the m-mode ansatz
 *     Psi = e^{i m phi~} r^3 Phi, the momentum Pi = d_t Phi + b d_r* Phi, the
 *     first-order system d_t u + D d_r* u = S with u = (Phi, Pi) complex,
 *     D = diag(b, -b) [d_matrix], and its two-step Lax-Wendroff iteration,
 *     half step (lw1) then full step (lw2), with second-order centred angular
 *     differences; boundary conditions Phi = Pi = 0 on both radial ends and,
 *     at the poles, d_theta Phi = 0 for even |m| or Phi = 0 for odd |m|.
 *   - The source term T of Eq. (1) is replaced by a Gaussian-smeared point
 *     particle F (the paper does not print T); F enters the Pi row of S and
 *     is produced by its own compact data-parallel pass over the cells near
 *     the orbit, as the paper produces T by its own kernel (Sec. 4).
 *
 * Conventions for every entry point:
 *   - Return 0 on success or a negative TEUK_E* code; teuk_last_error()
 *     then holds a message for the calling thread.  No C++ exception crosses
 *     this boundary.
 *   - Complex fields are complex128: interleaved (re, im) doubles, laid out
 *     [theta row j][r* column i], row-major, dense (row pitch = nr).
 *   - Pointers documented as "device" are HIP device pointers readable and
 *     writable on the context's stream; "host" pointers are ordinary memory.
 *     The caller owns every pointer it passes; the library never frees it and
 *     does not keep it after the call returns (except where stated).
 *   - Work is enqueued on the stream given to teuk_init_grid and runs
 *     asynchronously; calls that return host data synchronize that stream.
 *   - A context is not thread safe; use one context per host thread.
 *   - Device memory belongs to the caller.  A context lives in one
 *     caller-owned device workspace (teuk_workspace_size gives its size):
 *     the state (two time levels), the coefficient records, the source
 *     windows and, if requested, the adjoint's planes and partial sums.  The
 *     orbit table of a source and the snapshots of a checkpointed gradient go
 *     into further caller-owned device buffers named at those calls.  The
 *     library calls no device allocator; a buffer too small for what is asked
 *     of it is TEUK_ENOMEM, reported before any work is enqueued.  Every
 *     buffer must stay alive, unmoved, for as long as the context uses it
 *     (the workspace: until teuk_destroy).
 */
#ifndef TEUK_H
#define TEUK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TEUK_OK          0
#define TEUK_EINVAL     -1   /* invalid argument or descriptor            */
#define TEUK_EDEVICE    -2   /* HIP runtime error (message appended)      */
#define TEUK_ENONFINITE -3   /* non-finite values found by teuk_check_finite */
#define TEUK_ENOMEM     -4   /* a caller buffer is too small, or host memory ran out */
#define TEUK_ESTATE     -5   /* call order violated (e.g. no source set)  */

typedef struct teuk_ctx teuk_ctx;

/* Grid and physics of one instance.
 *   M, a      black-hole mass and spin, 0 <= |a| < M                 (Eq. 1)
 *   s, m      spin weight (-2..2) and azimuthal number              (Eq. 1, ansatz)
 *   nr, nth   nodes in r* and theta, both ends included: r*_i = rs_min + i h_r,
 *             h_r = (rs_max - rs_min)/(nr-1); theta_j = j h_th, h_th = pi/(nth-1);
 *             nr >= 5, 7 <= nth <= 65535
 *   cfl       dt = cfl * min(h_r, r(rs_min) h_th); 0 < cfl <= 1
 *   rs_extract extraction radius; the waveform is Phi at the nearest node
 *   ko_eps    strength of the theta fourth-difference dissipation added in the
 *             full step (0 = the literal scheme; 0 <= ko_eps <= 1).  The literal
 *             scheme is weakly unstable for stiff angular modes at the poles. */
typedef struct {
    double M, a;
    int32_t s, m;
    int32_t nr, nth;
    double rs_min, rs_max;
    double cfl;
    double rs_extract;
    double ko_eps;
} teuk_grid_desc;

/* Derived grid quantities (filled by teuk_get_info). */
typedef struct {
    double dt, h_r, h_th;
    double r_plus, r_minus;     /* horizons */
    int32_t i_ext;              /* extraction column */
    int32_t nr, nth;
    int32_t row_pitch;          /* internal row pitch of the state, in complex elements */
    int64_t steps_done;         /* iterations taken since the last teuk_set_state/teuk_init_pulse */
} teuk_info;

/* Synthetic point-particle source: F(t, r*, theta) = amplitude
 *   * G(r* - r*_p(t); sigma_r_cells h_r) * G(theta - theta_p(t); sigma_th_cells h_th)
 *   * exp(-i m phi~_p(t)),  G(x; s) = exp(-x^2/2s^2)/(sqrt(2 pi) s), zero where
 *   |x| > cutoff_sigmas * s.  The orbit is sampled at t_k = k dt/2,
 *   k = 0..nsamples-1: orbit[3k+0] = r*_p, orbit[3k+1] = theta_p,
 *   orbit[3k+2] = phi~_p (host array, read at the call).  Iteration n uses
 *   sample 2n in its half step (lw1, time t_n) and 2n+1 in its full step
 *   (lw2, time t_n + dt/2); stepping past the last sample is TEUK_ESTATE.
 *   orbit_dev: caller-owned device buffer of at least 3*nsamples doubles;
 *   teuk_set_source copies the orbit into it, and the source pass reads it
 *   there for as long as the source stays attached. */
typedef struct {
    double amplitude;
    double sigma_r_cells, sigma_th_cells, cutoff_sigmas;
    int64_t nsamples;
    const double* orbit;
    void* orbit_dev;
} teuk_source_desc;

/* What a context's workspace must hold besides the state and the
 * coefficient records.
 *   sigma_r_cells, sigma_th_cells, cutoff_sigmas  the largest source
 *        footprint the context will be given (teuk_source_desc); the source
 *        windows are sized for it.  All 0: no source.
 *   adjoint  nonzero: room for the reverse sweep (teuk_adjoint_*, and the
 *        checkpointed gradient): two more time levels and the dL/dA partial
 *        sums.
 * A NULL request means no source and no adjoint. */
typedef struct {
    double sigma_r_cells, sigma_th_cells, cutoff_sigmas;
    int32_t adjoint;
} teuk_ws_request;

/* Bytes of device workspace a context for (desc, req) needs (host output).
 * Validates the descriptor as teuk_init_grid does; touches no device. */
int teuk_workspace_size(const teuk_grid_desc* desc, const teuk_ws_request* req, size_t* bytes);

/* Create a context in the caller's workspace: validate the descriptor,
 * invert r*(r) (Newton on ln(r - r_+)), build the radial and angular
 * coefficient records of the first-order system on the host, copy them into
 * the workspace and zero the state.  dev_workspace: device memory of
 * ws_bytes bytes, 256-byte aligned (TEUK_EINVAL otherwise), at least
 * teuk_workspace_size bytes (TEUK_ENOMEM otherwise), owned by the caller and
 * kept alive until teuk_destroy.  hip_stream is a hipStream_t (NULL = the
 * null stream).  Synchronizes. */
int teuk_init_grid(const teuk_grid_desc* desc, const teuk_ws_request* req, void* hip_stream,
                   void* dev_workspace, size_t ws_bytes, teuk_ctx** out);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): teuk_init_grid with
 * the workspace taken from the library's own static device array of 64 MiB
 * (one per GPU, held until the process ends) instead of a caller's buffer.
 * Allocates no device memory: hipGetSymbolAddress finds the array once per
 * device; the context object itself and its host-side tables are ordinary
 * host memory.  At most one such context per device at a time (TEUK_ESTATE
 * while another holds it; teuk_destroy gives it back), so contexts cannot
 * overlap on one GPU; the array keeps the previous context's contents, and
 * the state planes are cleared at set-up.  TEUK_ENOMEM if
 * teuk_workspace_size(desc, req) exceeds 64 MiB (e.g. 6400 x 128 with a
 * source fits, with the adjoint area it does not).  Other arguments and
 * errors as teuk_init_grid. */
int teuk_init_grid_static(const teuk_grid_desc* desc, const teuk_ws_request* req, void* hip_stream,
                          teuk_ctx** out);

/* Release the context (host state and events); the workspace and every other
 * caller buffer stay with the caller.  Synchronizes the stream.  NULL is a
 * no-op. */
int teuk_destroy(teuk_ctx* ctx);

int teuk_get_info(const teuk_ctx* ctx, teuk_info* out);

/* Copy a state in (device, complex128 [nth][nr] each).  The values are taken
 * as given (no boundary projection).  Resets steps_done and the source clock. */
int teuk_set_state(teuk_ctx* ctx, const void* phi_dev, const void* pi_dev);

/* Copy the current state out (device, complex128 [nth][nr] each). */
int teuk_get_state(const teuk_ctx* ctx, void* phi_dev, void* pi_dev);

/* Initial data on the device: Phi = amplitude exp(-(r*-center)^2/(2 width^2)) P(theta),
 * P = 2^{(|m+s|+|m-s|)/2} sin^{|m+s|}(theta/2) cos^{|m-s|}(theta/2) (the lowest-l
 * spin-weighted profile), Pi = b d_r* Phi (time-symmetric data), then the
 * boundary conditions.  Resets steps_done and the source clock. */
int teuk_init_pulse(teuk_ctx* ctx, double center, double width, double amplitude);

/* Attach (or with NULL detach) the synthetic source.  Copies the orbit into
 * src->orbit_dev (TEUK_EINVAL if NULL) and keeps a host copy.  TEUK_ENOMEM if
 * the footprint is larger than the workspace was sized for (teuk_ws_request). */
int teuk_set_source(teuk_ctx* ctx, const teuk_source_desc* src);

/* Change the source amplitude without re-uploading the orbit. */
int teuk_set_amplitude(teuk_ctx* ctx, double amplitude);

/* Fill a host array with a circular equatorial prograde orbit sampled at
 * t_k = k dt/2, k = 0..nsamples-1: r*_p = r*(r0), theta_p = pi/2,
 * phi~_p = Omega t_k, Omega = M^{1/2}/(r0^{3/2} + a M^{1/2}).  out has 3*nsamples doubles. */
int teuk_orbit_circular(double M, double a, double r0, double dt, int64_t nsamples, double* out);

/* Fill a host array with a bound prograde equatorial Kerr geodesic of
 * semi-latus rectum p and eccentricity e (r = p/(1 + e cos chi), chi = 0 at
 * periapsis, chi = chi0 at t = 0), sampled at t_k = k dt/2,
 * k = 0..nsamples-1: r*_p, theta_p = pi/2, and phi~_p with phase zero at
 * t = 0 (d phi~ = d phi + a/Delta dr, the azimuth of Sec. 3.2).  The orbit
 * is the input of the synthetic source, which stands in for the paper's T.
 * E and L are closed-form; t(chi) and phi(chi) are cosine series of the
 * geodesic rates (accurate to rounding for e <= 0.9), inverted by Newton's
 * method.  TEUK_EINVAL for |a| >= M, e outside [0, 0.9], dt <= 0, or p and
 * e with no bound stable prograde orbit.  out has 3*nsamples doubles. */
int teuk_orbit_eccentric(double M, double a, double p, double e, double chi0, double dt, int64_t nsamples,
                         double* out);

/* Take nsteps iterations (lw1, boundary rows of the half step, lw2 with the
 * source and dissipation, boundary conditions).  If waveform_dev is not NULL
 * it receives nsteps*nth complex128: row n is Phi at the extraction column
 * after iteration n+1 of this call.  Asynchronous. */
int teuk_step_n(teuk_ctx* ctx, int64_t nsteps, void* waveform_dev);

/* ---- Adjoint (reverse sweep) -------------------------------------------
 * The iteration is C-linear, so the gradient of a real loss L, written as
 * dL/dRe + i dL/dIm, propagates as lambda^n = G^H lambda^{n+1}: the
 * conjugate transpose of one iteration, sub-step by sub-step (boundary
 * conditions, full step with dissipation, half-step pole rows, half step).
 * The waveform enters as lambda^n += dL/dw_n at the extraction column
 * (E^H), the source amplitude as dL/dA += sum_n Re<lambda, d u/dA>.
 *
 * gw_dev (device, may be NULL) holds dL/dw_n for the forward run, laid out as
 * the forward waveform: row n-1 = dL/dw_n (nth complex128), n = 1..n_end.
 *
 * teuk_adjoint_begin: lambda := (lam_phi, lam_pi) (device [nth][nr]; NULL = 0)
 *   plus dL/dw_{n_end} at the extraction column; the reverse clock is set to
 *   n_end (the forward iteration count lambda belongs to); dL/dA := 0.
 * teuk_adjoint_step_n: nsteps reverse iterations m = clock-1 .. clock-nsteps,
 *   each lambda := G^H lambda, then + dL/dw_m (m >= 1); with a source
 *   attached, accumulates dL/dA with the unit-amplitude source of forward
 *   iteration m.  Asynchronous.
 * teuk_adjoint_add_state: lambda += (gphi, gpi) (device [nth][nr]; NULL
 *   skips) - gradients of losses on the state at the current clock.
 * teuk_adjoint_get: copies lambda out (device, NULL skips) and, if dL_dA is
 *   not NULL, synchronizes and stores dL/dA there (host). */
int teuk_adjoint_begin(teuk_ctx* ctx, const void* lam_phi_dev, const void* lam_pi_dev, int64_t n_end,
                       const void* gw_dev);
int teuk_adjoint_step_n(teuk_ctx* ctx, int64_t nsteps, const void* gw_dev);
int teuk_adjoint_add_state(teuk_ctx* ctx, const void* gphi_dev, const void* gpi_dev);
int teuk_adjoint_get(teuk_ctx* ctx, void* lam_phi_dev, void* lam_pi_dev, double* dL_dA);

/* ---- Checkpointed gradient -----------------------------------------------
 * A loss may depend on states the caller does not keep:
 *   L_s = state_weight * sum_{n = n_lo..n_hi} sum_{j0 <= j < j1, i0 <= i < i1} |Phi^n_ij|^2.
 * Its reverse sweep needs Phi^n at every n in [n_lo, n_hi].  The iteration
 * is linear, so the reverse sweep needs no other forward state.  Two
 * schedules keep what it needs:
 *   snapshots = 0 (uniform): the forward keeps one snapshot of (Phi, Pi)
 *     every `interval` iterations (0 picks ceil(sqrt(nsteps))) and the
 *     backward recomputes each segment from its snapshot once, keeping Phi
 *     on the rectangle, before sweeping it in reverse.  One forward
 *     recompute in all; memory nsteps/interval snapshots plus `interval`
 *     copies of the rectangle.
 *   snapshots = s >= 1 (binomial, for a memory budget): at most s snapshots
 *     of (Phi, Pi) are held at any time, placed by the binomial schedule of
 *     teuk_checkpoint_schedule (Griewank's revolve); reversing nsteps
 *     iterations then recomputes r*nsteps - C(s + r, s + 1)
 *     forward iterations, r the smallest number with C(s + r, s) >= nsteps.
 *     `interval` must be 0.
 * With state_weight = 0 the states are not needed; force_recompute != 0
 * runs the schedule's recomputation anyway (same gradient, bitwise).
 *
 * The snapshots, the rectangle buffer and the loss's partial sums live in
 * the caller-owned device buffer ckpt_dev of ckpt_bytes bytes, 256-byte
 * aligned, at least teuk_checkpoint_size(plan) (TEUK_ENOMEM otherwise); it
 * must stay alive from the forward through the backward.  The context's
 * workspace must have the adjoint area (teuk_ws_request.adjoint).
 *
 * teuk_forward_checkpointed: from the state set by teuk_set_state or
 *   teuk_init_pulse (no iteration taken since), runs plan->nsteps
 *   iterations, writing the waveform (device, may be NULL) as teuk_step_n
 *   does, and, if state_loss is not NULL, stores L_s there (host;
 *   synchronizes).
 * teuk_backward_checkpointed: right after the forward with the same plan,
 *   takes dL/dw (gw_dev, forward waveform layout, may be NULL) and dL/dL_s,
 *   and writes dL/dPhi^0, dL/dPi^0 (device [nth][nr]) and dL/dA (host, may
 *   be NULL; synchronizes).  The forward state is left at an intermediate
 *   iteration afterwards. */
typedef struct {
    int64_t nsteps;
    int64_t interval;
    int64_t snapshots;
    double state_weight;
    int32_t i0, i1, j0, j1;
    int64_t n_lo, n_hi;
    int32_t force_recompute;
    void* ckpt_dev;
    uint64_t ckpt_bytes;
} teuk_grad_plan;

/* Bytes of checkpoint buffer (plan->ckpt_dev) the plan needs (host output);
 * ckpt_dev and ckpt_bytes are not read. */
int teuk_checkpoint_size(const teuk_ctx* ctx, const teuk_grad_plan* plan, size_t* bytes);

/* The binomial schedule for nsteps >= 1 iterations and snapshots >= 1
 * slots (host only: needs no device or context).  phase 0 lists the
 * forward's actions (from u^0 to u^nsteps), phase 1 the backward's (from
 * u^nsteps down to reverse iteration 0), as triples (op, a, b) of int64:
 *   op 0  advance a iterations from the current state, reaching iteration b;
 *   op 1  store the current state u^b in slot a;
 *   op 2  restore slot a, which holds u^b, into the current state;
 *   op 3  reverse iteration a (lambda^{a+1} -> lambda^a) with the current
 *         state at u^a.
 * *count receives the number of actions of the phase; the first
 * min(*count, cap) are written to actions (3 * cap int64, may be NULL with
 * cap 0).  stats (may be NULL) receives {r, forward iterations recomputed by
 * the backward, largest number of slots held at once}.  EINVAL for
 * nsteps < 1, snapshots < 1 or phase not 0 or 1. */
int teuk_checkpoint_schedule(int64_t nsteps, int64_t snapshots, int32_t phase, int64_t* actions, int64_t cap,
                             int64_t* count, int64_t* stats);

int teuk_forward_checkpointed(teuk_ctx* ctx, const teuk_grad_plan* plan, void* waveform_dev,
                              double* state_loss);
int teuk_backward_checkpointed(teuk_ctx* ctx, const teuk_grad_plan* plan, const void* gw_dev,
                               double dL_dLs, void* grad_phi0_dev, void* grad_pi0_dev, double* dL_dA);

/* Current Phi column at the extraction radius: nth complex128 (device). */
int teuk_extract_waveform(const teuk_ctx* ctx, void* out_dev);

/* Synchronize and check that the state is finite; TEUK_ENONFINITE if not. */
int teuk_check_finite(teuk_ctx* ctx);

/* Launch configuration of the stencil (results are bitwise identical for
 * every valid setting; only speed changes).
 *   seg_rows  theta rows per wave segment of the streaming stencil.
 *   k_steps   iterations per launch (temporal blocking).  1: the single-step
 *             kernel, seg_rows 4, 8 or 16.  k > 1: the blocked kernel runs k
 *             consecutive iterations (half and full steps, boundary rows,
 *             source and extraction of each) in one launch, reading u^n from
 *             and writing u^{n+k} to HBM once; (seg_rows, k_steps) one of
 *             (4, 2), (8, 2), (4, 4).  teuk_step_n runs floor(nsteps / k)
 *             blocks and the remainder as single iterations.
 *   adj_seg_rows  theta rows per wave segment of the adjoint kernel
 *             (teuk_adjoint_step_n), 4, 8 or 16; 0 in teuk_set_tuning leaves
 *             it unchanged.  Default 16 where 16-row segments give more
 *             waves than the device has SIMDs, else 4 (teuk_autotune does
 *             not change it).
 * The default (k_steps 1, seg_rows from the grid size) is set by
 * teuk_init_grid; teuk_autotune chooses (seg_rows, k_steps) by measurement.
 * EINVAL for any other values. */
typedef struct {
    int32_t seg_rows;
    int32_t k_steps;
    int32_t adj_seg_rows;
} teuk_tuning;

int teuk_set_tuning(teuk_ctx* ctx, const teuk_tuning* t);
int teuk_get_tuning(const teuk_ctx* ctx, teuk_tuning* out);

/* Autotuner over the launch configurations above.
 * Times every valid (seg_rows, k_steps) pair on this context's grid with HIP
 * events (warm-up, then the best of three timed runs of a fixed number of
 * iterations, without extraction, with the context's source when its orbit
 * table covers the 624 trial iterations from the current one, else without),
 * keeps the fastest as the context's tuning, and leaves the state,
 * iteration count and source as they were (the state is saved to and
 * restored from host memory; synchronizes the stream).
 *   cache_path  host string or NULL.  A text file of lines
 *               "<key>\t<seg_rows>\t<k_steps>\t<us per iteration>", where the
 *               key names the device architecture, nr, nth, whether a != 0,
 *               whether the dissipation is on, whether the trials ran with
 *               the source, and a hash of the kernel sources the library
 *               was built from.  If a line with this
 *               context's key exists its pair is applied without measuring;
 *               otherwise the measured choice is appended (the file is
 *               created if missing).  Unreadable/unwritable file: EINVAL.
 *   table       host array of capacity entries or NULL: receives every
 *               measured pair (or the one cached pair), fastest first;
 *               *count (host, may be NULL) = entries written.
 * ENOMEM if the host copy of the state cannot be allocated. */
typedef struct {
    int32_t seg_rows;
    int32_t k_steps;
    int32_t batch_mode;     /* batches: TEUK_BATCH_*; 0 for a single context */
    double us_per_iteration;
} teuk_tune_entry;

int teuk_autotune(teuk_ctx* ctx, const char* cache_path, teuk_tune_entry* table, int32_t capacity,
                  int32_t* count);

#define TEUK_BATCH_PERSISTENT 0
#define TEUK_BATCH_PER_ITERATION 1

/* Batched stepping: many independent instances (each its own M, a, s, m,
 * grid and state) advanced together, in one of two modes.
 * TEUK_BATCH_PERSISTENT: ONE persistent kernel launch per call, captured in
 *   a HIP graph together with a small kernel that resets its work counters.
 *   Work items are tiles (instance, strip of 62 r* columns over all theta
 *   rows, walked in segments of seg_rows rows) of one iteration; persistent
 *   waves take them from a global counter in iteration-major order, and each
 *   item waits on per-tile completion counters of its neighbouring strips
 *   (the iteration's data dependences, Sec. 3.2 half and full steps) instead
 *   of a launch boundary.
 * TEUK_BATCH_PER_ITERATION: one launch per iteration covering every
 *   instance, one wave per (instance, strip, theta segment); the launch
 *   boundary orders the iterations.  When the instances' two state levels
 *   together exceed 256 MiB (the last-level cache), the instances are
 *   packed into groups of at most 96 MiB per level (first fit, largest
 *   first; an instance larger than that is a group of its own), and each
 *   group runs a whole chunk of iterations (up to 256) before the next, one
 *   launch per iteration over the group, so that its levels stay in the
 *   cache.  The order of work changes, not the arithmetic.
 * Every point is evaluated by the same device code as teuk_step_n, so an
 * instance's results are bitwise equal to stepping it alone, in both modes.
 *
 * teuk_batch_workspace_size: bytes of device workspace for a batch of n
 *   instances (host output): the batch's own tables (instance table, tiles,
 *   item offsets, completion counters, work counter, abort flag) followed by
 *   one context workspace per instance, every instance with request req
 *   (NULL: no source, no adjoint).  Touches no device.
 * teuk_batch_create: n >= 1 descriptors (host array); every instance gets a
 *   context as from teuk_init_grid on hip_stream, in its part of the
 *   caller's workspace (dev_workspace, ws_bytes: 256-byte aligned, at least
 *   teuk_batch_workspace_size; kept alive until teuk_batch_destroy).
 *   Validation as there; the message names the failing instance.  The
 *   instance tables are staged through two small pinned host buffers.
 *   Synchronizes.
 * teuk_batch_instance: borrowed context of instance k (0 <= k < n), for
 *   teuk_set_state / teuk_init_pulse / teuk_get_state / teuk_step_n / ...;
 *   teuk_destroy refuses it (EINVAL), teuk_batch_destroy frees it.
 * teuk_batch_set_tuning / get_tuning: theta rows per segment, 4, 8 or 16
 *   (EINVAL otherwise); synchronizes.  The default is 16.
 * teuk_batch_set_mode / get_mode: TEUK_BATCH_PER_ITERATION (the default,
 *   the faster mode on every batch measured) or TEUK_BATCH_PERSISTENT
 *   (EINVAL otherwise); applies from the next teuk_batch_step_n.
 * teuk_batch_get_groups: the per-iteration mode's groups, fixed at
 *   teuk_batch_create.  *ngroups: their number (1 when the batch fits the
 *   cache).  first: NULL or a host array of ngroups + 1 entries, receiving
 *   the first device-table position of each group and then n.  order: NULL
 *   or a host array of n entries, receiving the instances (the caller's
 *   indices k) in device-table order, group by group, ascending within a
 *   group (the identity when there is one group).  EINVAL for a null
 *   ngroups.
 * teuk_batch_step_n: nsteps (0 <= nsteps <= INT32_MAX) iterations of every
 *   instance.  waveforms = NULL or a host array of n device pointers, each
 *   NULL or nsteps * nth complex128 (the extraction column after every
 *   iteration, as teuk_step_n).  Instances may carry sources (teuk_set_source
 *   on the instance: e.g. every m of one orbit, or an inspiralling orbit
 *   table); then the iterations go in chunks of at most 256, each preceded by
 *   the compact source pass of every instance that has one, exactly as
 *   teuk_step_n would run it.  ESTATE if an instance's orbit has too few
 *   samples for nsteps more iterations (nothing is launched).  Asynchronous;
 *   in the persistent mode the graph for (rounds, seg_rows) is captured on
 *   first use and cached.
 * teuk_batch_sync: synchronizes the stream and reports a persistent launch
 *   that gave up (TEUK_EDEVICE): a dependency wait that exceeds 2 s of device
 *   wall clock
 *   makes every wave of that launch, and of launches queued after it, exit
 *   early, leaving the states invalid.  Reading the report clears it.
 * teuk_batch_autotune: as teuk_autotune over (batch_mode, seg_rows)
 *   (k_steps is 1 for batches), timing 8 batched iterations per variant with
 *   sources detached, all instance states, clocks and sources restored
 *   afterwards; applies the fastest mode and
 *   segment length.  Cache lines carry a fifth column, the mode; cache key
 *   = architecture, the instance shapes and the kernel sources. */
typedef struct teuk_batch teuk_batch;

int teuk_batch_workspace_size(int32_t n, const teuk_grid_desc* descs, const teuk_ws_request* req, size_t* bytes);
int teuk_batch_create(int32_t n, const teuk_grid_desc* descs, const teuk_ws_request* req, void* hip_stream,
                      void* dev_workspace, size_t ws_bytes, teuk_batch** out);
int teuk_batch_destroy(teuk_batch* batch);
int teuk_batch_instance(teuk_batch* batch, int32_t k, teuk_ctx** out);
int teuk_batch_set_tuning(teuk_batch* batch, int32_t seg_rows);
int teuk_batch_get_tuning(const teuk_batch* batch, int32_t* seg_rows);
int teuk_batch_set_mode(teuk_batch* batch, int32_t mode);
int teuk_batch_get_mode(const teuk_batch* batch, int32_t* mode);
int teuk_batch_get_groups(const teuk_batch* batch, int32_t* ngroups, int32_t* first, int32_t* order);
int teuk_batch_step_n(teuk_batch* batch, int64_t nsteps, void* const* waveforms);
int teuk_batch_sync(teuk_batch* batch);

/* Bounded waits of the persistent mode.
 * teuk_batch_set_wait_limit: device wall-clock time a dependency wait may
 *   take before the launch gives up (sets the abort flag; every wave then
 *   leaves at the top of its next pass), 0 <= seconds <= 3600, default 2.
 *   Synchronizes; drops the captured graphs (the limit is a launch
 *   argument).  0 makes every wait that is not satisfied at its first check
 *   give up.
 * teuk_batch_abort: enqueues on the batch's stream a store of the abort
 *   flag, so that persistent launches queued after it exit at their first
 *   pass (per-iteration launches do not look at it).  teuk_batch_sync then
 *   reports TEUK_EDEVICE once and clears the flag.  For cancelling queued
 *   persistent work, and for testing the abort path without a broken
 *   dependency. */
int teuk_batch_set_wait_limit(teuk_batch* batch, double seconds);
int teuk_batch_abort(teuk_batch* batch);
int teuk_batch_autotune(teuk_batch* batch, const char* cache_path, teuk_tune_entry* table, int32_t capacity,
                        int32_t* count);

/* Measurement aid: while enabled, every stencil launch made by teuk_step_n
 * records a pair of HIP events at the start and end of that kernel's
 * execution (hipExtLaunchKernel; the source pass is not timed).
 * teuk_kernel_timing synchronizes and returns the summed kernel time (ms)
 * and the number of timed launches since timing was enabled.  Enabling
 * resets the sums. */
int teuk_set_kernel_timing(teuk_ctx* ctx, int enable);
int teuk_kernel_timing(teuk_ctx* ctx, double* total_ms, int64_t* launches);

/* ---- Radiated energy and momentum -----------------------------------------
 * The waves carry energy, linear and angular momentum away from the binary,
 * which recoils (Sec. 3.2, closing paragraph, and its figure of the kick).
 * From the extracted waveforms of several m modes of one system (Phi at the
 * extraction column, which stands for r psi_4 at large r: for s = -2,
 * Psi = rho^-4 psi_4 and Psi = e^{i m phi~} r^3 Phi), with the news integral
 * H_m = int_0^t Phi_m dt' and K_m = int_0^t H_m dt' (trapezoidal rule):
 *   dE/dt           = 1/2 sum_m int |H_m|^2 sin dtheta
 *   d(Px + i Py)/dt = 1/2 sum_m int H_m conj(H_{m+1}) sin^2 dtheta
 *   dPz/dt          = 1/2 sum_m int |H_m|^2 cos sin dtheta
 *   dJz/dt          = 1/2 sum_m m Im int conj(H_m) K_m sin dtheta
 * (the standard psi_4 flux integrals over the sphere, their phi integrals
 * done exactly on the Fourier modes; theta integrals by the trapezoidal
 * rule on the rows theta_j = j pi/(nth - 1)).
 *   nmodes  1..16 waveforms; m (host array) their azimuthal numbers, distinct;
 *   waves   host array of nmodes device pointers, each (nsteps + 1) x nth
 *           complex128: row n = Phi at the extraction column at t = n dt
 *           (row 0 the initial state: teuk_extract_waveform before stepping,
 *           then the rows teuk_step_n writes);
 *   out_dev (nsteps + 1) x 10 doubles (device): dE/dt, dPx/dt, dPy/dt,
 *           dPz/dt, dJz/dt, then E, Px, Py, Pz, Jz accumulated from t = 0 by
 *           the trapezoidal rule (the recoil velocity is -P/M).
 * The running integrals go into the caller's dev_workspace (ws_bytes, at
 * least teuk_flux_workspace_size, 256-byte aligned).  Asynchronous on
 * hip_stream. */
typedef struct {
    int32_t nmodes;
    const int32_t* m;
    const void* const* waves;
    int64_t nsteps;
    int32_t nth;
    double dt;
} teuk_flux_desc;

int teuk_flux_workspace_size(const teuk_flux_desc* desc, size_t* bytes);
int teuk_radiated_flux(const teuk_flux_desc* desc, void* hip_stream, void* dev_workspace, size_t ws_bytes,
                       void* out_dev);

/* Message for the last failed call on this thread ("" if none). */
const char* teuk_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TEUK_H */
