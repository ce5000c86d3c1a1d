/*
 * specstep.h -- C ABI of the MI355X (gfx950) semi-implicit Fourier spectral
 * step library (libspecstep.so).
 *
 * The method (Sec. 2.4.2 of Silber & Karttunen, "SymPhas -- general purpose
 * software for phase-field, phase-field crystal and reaction-diffusion
 * simulations"): an equation of motion d psi/dt = L{psi} + sum_i N_i{f_i(psi)}
 * (Eq. 1) is Fourier transformed (Eq. 2) and advanced per wavevector by
 *     psi^(t+dt) = A psi^(t) + B sum_i N_i f_i^(psi(t)),
 *     A = exp(L dt),  B = (exp(L dt) - 1)/L                     (Eqs. 3, 4)
 * with A and B computed once per model and time step (Sec. 2.4.2) and the
 * nonlinear terms evaluated pointwise in real space every step.  Periodic
 * boundaries are implied by the transform (Sec. 2.4.2).  Grids are
 * row-major with x the fastest axis (Sec. 2.2.1).
 *
 * Conventions shared by every entry point
 *   - Every call returns an ss_status and never throws or exits.  On an
 *     error the thread-local message is available from ss_last_error().
 *   - The library never allocates device memory: the caller provides the
 *     workspace (ss_bind_workspace) and the mass log buffer.  Handles are
 *     created by ss_create_grid and freed by ss_destroy_grid.
 *   - Device work is enqueued on the HIP stream given at creation
 *     (ss_set_stream to change it).  ss_step_n never synchronises; calls
 *     that read or write host memory synchronise the stream before they
 *     return.  Host pointers are only read/written during the call.
 *   - Field arrays are C-contiguous (nz, ny, nx) arrays of the grid's
 *     element type (float for SS_F32, double for SS_F64), x fastest.
 *   - Launch failures return SS_ERR_DEVICE; faults of earlier asynchronous
 *     work surface at a later call.
 */
#ifndef SPECSTEP_H
#define SPECSTEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ss_grid_s* ss_grid;

typedef enum {
  SS_OK = 0,
  SS_ERR_ARG = 1,          /* invalid argument (null, range, non-finite) */
  SS_ERR_UNSUPPORTED = 2,  /* valid but not implemented (e.g. axis not 2^k) */
  SS_ERR_STATE = 3,        /* call out of order (no model, workspace, field) */
  SS_ERR_DEVICE = 4,       /* HIP runtime error */
  SS_ERR_NONFINITE = 5     /* ss_check_finite found a NaN or an infinity */
} ss_status;

typedef enum { SS_F32 = 4, SS_F64 = 8 } ss_dtype;

/* Models and their coefficient vectors (Sec. 3, Eqs. 9-13; Gray-Scott
 * reaction-diffusion is named in Sec. 1 but not written out).
 *   SS_ALLEN_CAHN    {M, kappa, c1, c2}   d psi/dt = M (kappa lap psi + c1 psi - c2 psi^3)
 *   SS_CAHN_HILLIARD {M, kappa, c1, c2}   d psi/dt = M lap (c2 psi^3 - c1 psi - kappa lap psi)
 *   SS_PFC           {r, q0, g2, g3}      d psi/dt = lap[(r + (q0^2 + lap)^2) psi + g2 psi^2 + g3 psi^3]
 *   SS_GRAY_SCOTT    {Du, Dv, F, k}       u_t = Du lap u - u v^2 + F (1 - u)
 *                                         v_t = Dv lap v + u v^2 - (F + k) v   (fields 0 = u, 1 = v)
 *   SS_MODEL_C       {c1, c2, c3, c4, c5} psi_t = lap psi + c1 psi - c2 psi^3 + 2 c5 psi m
 *                                         m_t = -lap^2 m - lap(c3 m - c4 m^3 + c5 psi^2)  (0 = psi, 1 = m)
 * Every term linear in a field goes into L (solved exactly by A); the
 * remaining terms are the explicit f_i. */
typedef enum {
  SS_ALLEN_CAHN = 1,
  SS_CAHN_HILLIARD = 2,
  SS_PFC = 3,
  SS_GRAY_SCOTT = 4,
  SS_MODEL_C = 5,
  SS_EQUATIONS = 6      /* equations read at run time: set by ss_set_equations only */
} ss_model;

/* Create a grid handle.  ndim is 2 or 3; n[0] is the x extent (fastest),
 * n[1] y, n[2] z; each a power of two in [8, 4096] (3D: z <= 1024).
 * dx[] are the spacings (> 0, finite), same order.  stream is a
 * hipStream_t (NULL = default stream).  The wavenumbers are
 * k_j = 2 pi m_j / (n_j dx_j) (Sec. 2.4.2).
 * Errors: SS_ERR_ARG, SS_ERR_UNSUPPORTED. */
ss_status ss_create_grid(int ndim, const int64_t n[], const double dx[], ss_dtype dtype,
                         void* stream, ss_grid* out);

/* Choose the model, its coefficients (ncoef as listed above) and the time
 * step dt > 0.  Plays the role of the solver's one-time set-up that forms
 * the A and B operators a priori (Sec. 2.2.4, Sec. 2.4.2).  Changing the
 * model drops the bound workspace and fields (SS_ERR_STATE afterwards
 * until they are bound/set again); changing only coef or dt keeps them.
 * Errors: SS_ERR_ARG (unknown model, ncoef, non-finite, dt <= 0). */
ss_status ss_set_model(ss_grid g, ss_model model, const double* coef, int ncoef, double dt);

/* ---- Equations read at run time ---------------------------------------------
 * The spectral scheme built from an equation of motion given as text
 * (Sec. 2.4.2: the procedure that splits any equation into the linear
 * operator, giving A, and derivative-grouped explicit terms, giving the
 * B_i and E_i; the update psi^' = A psi^ + sum_i B_i (E_i^0 + E_i^1)^).
 *
 * Text: one equation per field (1 or 2 fields, in the order given, which
 * is the field index), separated by ';' or newlines, each
 *     name' = expression
 * with numbers (decimal, optional exponent), the coefficient names of
 * names[] (values[] holds their values), field names, + - * /, '^' or '**'
 * with an integer literal exponent 0..16, parentheses, lap(e) and bilap(e)
 * = lap(lap(e)); parentheses, lap/bilap and unary signs nested at most
 * 200 deep.  Division only by constant expressions.  Example
 * (Cahn-Hilliard):  "psi' = M*lap(c2*psi^3 - c1*psi - kappa*lap(psi))".
 *
 * The right-hand side is expanded into terms c lap^p (monomial in the
 * fields).  Terms linear in the field itself form L (symbol lap -> -|k|^2,
 * at most lap^3, so L(k^2) is at most cubic in k^2).  All other terms --
 * constants, terms in the other field, nonlinear terms -- are explicit and
 * are evaluated pointwise from the fields of the current step; the explicit
 * terms under the same derivative lap^p form one channel i with operator
 * B_i = B (-k^2)^p (Sec. 2.4.2, the pairing of L_* and N terms by
 * derivative).  Limits of the GPU step: at most two channels per field,
 * p <= 3, each with at most 8 monomials with exponents at most 7 (a
 * second channel costs one more forward transform and one more array per
 * field: the workspace grows by nfields arrays); the finite-difference
 * solver takes one channel per field.  A derivative multiplied by a field
 * (psi lap psi) has no operator form and is refused.
 *
 * scheme 0: ETD1 factors A = exp(L dt), B = (exp(L dt) - 1)/L (Eq. 4).
 * scheme 1: linearly implicit factors A = 1/(1 - L dt), B = dt/(1 - L dt),
 *   the first-order semi-implicit scheme; requires L(k^2) dt < 1 for all
 *   k^2 up to the grid's largest, sum_a (pi/dx_a)^2.
 * Afterwards the grid behaves as with ss_set_model (model SS_EQUATIONS):
 * ss_step_n, fields, mass log, structure factor, autotune and timing work;
 * the adjoint and batches are SS_ERR_UNSUPPORTED.  With the
 * finite-difference solver (ss_set_solver, before or after) the same split
 * is stepped by forward Euler (Sec. 2.4.1): psi_j += dt (sum_p c_p lap^p
 * psi_j + lap^p_j E_j), every Laplacian the chosen stencil; scheme must
 * be 0 there.  Replacing equations with the same number of fields
 * keeps the workspace and fields (like changing coefficients); otherwise
 * they are dropped.
 * Errors: SS_ERR_ARG (unreadable text, unknown or duplicate names,
 * non-finite values, dt <= 0, unknown scheme, 1 - L dt <= 0),
 * SS_ERR_UNSUPPORTED (a valid equation outside the limits above, or
 * scheme 1 with the finite-difference solver). */
ss_status ss_set_equations(ss_grid g, const char* equations, const char* const names[],
                           const double values[], int nvalues, double dt, int scheme);

/* Host-only: the split ss_set_equations performs, without a grid or a
 * device.  out (at least SS_SPLIT_OUT_LEN doubles) receives out[0] = the
 * number of fields and, for field j at o = out + 1 + SS_SPLIT_FIELD_LEN j:
 * o[0..3] = the coefficients of L in 1, k^2, k^4, k^6; o[4] = the number
 * of explicit channels (0, 1 or 2, in ascending derivative order); channel
 * c at q = o + 5 + SS_SPLIT_CHANNEL_LEN c: q[0] = p, its derivative lap^p;
 * q[1] = m, its number of monomials; then for i < m: q[2 + 3i] =
 * coefficient, q[3 + 3i], q[4 + 3i] = the exponents of fields 0 and 1.
 * Unused entries are 0.
 * Errors: as ss_set_equations (no grid checks). */
#define SS_SPLIT_CHANNEL_LEN 26
#define SS_SPLIT_FIELD_LEN (5 + 2 * SS_SPLIT_CHANNEL_LEN)
#define SS_SPLIT_OUT_LEN (1 + 2 * SS_SPLIT_FIELD_LEN)
ss_status ss_split_equations(const char* equations, const char* const names[], const double values[],
                             int nvalues, double* out, int nout);

/* ---- Solver choice ---------------------------------------------------------
 * solver 0 (default): the semi-implicit spectral scheme (Sec. 2.4.2).
 * solver 1: explicit forward Euler with finite differences (Sec. 2.4.1):
 *   q <- q + dt * rhs(q) on the real-space fields, the right-hand sides of
 *   the models above, or of the equations of ss_set_equations, with the
 *   Laplacian replaced by a finite-difference stencil
 *   (Sec. 2.2.2; periodic wrap; higher powers by composition):
 *   stencil 0 (or 5 in 2D, 7 in 3D): axis-wise central differences,
 *   sum_a (f[-1] - 2 f + f[+1]) / dx_a^2;  stencil 4: the fourth-order
 *   axis-wise stencil (fourth-order family, 9 points in 2D, 13 in 3D),
 *   sum_a (-f[-2] + 16 f[-1] - 30 f + 16 f[+1] - f[+2]) / (12 dx_a^2).
 *   The isotropic stencils need equal spacings h (faces / edges / corners:
 *   the neighbours at distance 1 / sqrt 2 / sqrt 3; A1, A2 the axis ones at
 *   1 and 2, D1, D2 the diagonal ones at (1, 1) and (2, 2), K the 8 at
 *   (1, 2) and (2, 1)), second order:
 *     9 (2D):  (4 edges + corners - 20 centre) / (6 h^2);
 *     15 (3D): (8 faces + corners - 56 centre) / (12 h^2);
 *     19 (3D): (2 faces + edges - 24 centre) / (6 h^2);
 *     21 (3D): (4 edges - corners - 40 centre) / (12 h^2) (its symbol is
 *              +4/(3 h^2) at the checkerboard mode: explicit diffusion
 *              with it amplifies that mode);
 *     27 (3D): (14 faces + 3 edges + corners - 128 centre) / (30 h^2);
 *   fourth order (2D only):
 *     17: (128 A1 + 16 D1 - 8 A2 - D2 - 540 centre) / (120 h^2);
 *     21: (52 A1 + 16 D1 - A2 - 2 K - 252 centre) / (60 h^2).
 *   Sec. 2.2.2 names these point counts; the weights are those its
 *   families' defining conditions fix on each point set (zero sum, second
 *   moment 2 per axis, an error term that depends on |k| only: h^2 |k|^4
 *   / 12 for second order, h^4 |k|^6 / 90 for fourth order).
 *   Explicit: stable only for dt below the stencil's limit (the caller's
 *   choice).  The fields live in real space; ss_set_field / ss_get_field /
 *   ss_step_n work as with the spectral solver; the mass log is not
 *   written; ss_step_n_profiled, ss_time_pass, ss_autotune,
 *   ss_structure_factor, the adjoint and batches are SS_ERR_UNSUPPORTED.
 * Changing the solver drops the bound workspace and fields (its size
 * differs: (2 nfields + 3) arrays for solver 1).
 * Errors: SS_ERR_ARG (unknown solver or stencil for the dimension),
 * SS_ERR_UNSUPPORTED (isotropic stencil with unequal spacings; solver 1
 * for equations set with scheme 1). */
ss_status ss_set_solver(ss_grid g, int solver, int stencil);

/* Kernel that advances the spectral step (results agree to rounding).
 * kind 0: the pass kernels, two launches per step (every grid).
 * kind 1: one workgroup runs all the steps of a call of ss_step_n: the
 *   spectral state of the grid stays in its registers and LDS between
 *   steps (no launch, no HBM traffic per step) and the per-mode factors
 *   A and B N are computed once per call into the grid's scratch and
 *   staging arrays.  For the small grids on which the pass kernels are
 *   latency-bound: 2D square grids of 16, 32, 64 or 128 points a side, one
 *   field, the fixed models (SS_ALLEN_CAHN, SS_CAHN_HILLIARD, SS_PFC),
 *   spectral solver.  The mass log is written as with kind 0.
 * ss_autotune (while no field is stored) times both and keeps the faster
 * unless ss_set_step_kernel chose; ss_get_step_kernel reports the kind
 * ss_step_n uses.  ss_step_n_profiled, ss_time_pass and
 * ss_step_fields_noalloc use the pass kernels.
 * Errors: SS_ERR_ARG (kind), SS_ERR_STATE (no model), SS_ERR_UNSUPPORTED
 * (kind 1 for another grid). */
ss_status ss_set_step_kernel(ss_grid g, int kind);
ss_status ss_get_step_kernel(ss_grid g, int* kind);

/* Bytes of device workspace the grid needs (after ss_set_model or
 * ss_set_equations): for the spectral solver (3 nfields + 1) arrays of
 * nx*ny*nz reals -- per field the partly transformed state, its full
 * spectrum (carried between steps so that a step transforms the state only
 * once, inversely) and a scratch array (the transformed nonlinear term
 * unless the step runs in place, see ss_set_step_arrangement), plus one
 * staging array; for the finite-difference solver (2 nfields + 3). */
ss_status ss_workspace_size(ss_grid g, size_t* bytes);

/* Bind caller-owned device memory of at least ss_workspace_size bytes,
 * 256-byte aligned.  The library keeps the pointer; the caller keeps it
 * alive until the handle is destroyed or rebound and the work already
 * enqueued on the grid's stream has finished (neither waits for it).
 * Errors: SS_ERR_STATE (no model), SS_ERR_ARG (null, too small, misaligned). */
ss_status ss_bind_workspace(ss_grid g, void* device_ptr, size_t bytes);

/* Load field `field` (0 .. nfields-1) from src, a (nz, ny, nx) array of
 * the grid dtype on the device (src_on_device = 1) or the host (0).
 * Errors: SS_ERR_STATE (no workspace), SS_ERR_ARG, SS_ERR_DEVICE. */
ss_status ss_set_field(ss_grid g, int field, const void* src, int src_on_device);

/* Write field `field` in real space to dst (device or host, as above).
 * Errors: SS_ERR_STATE (field never set), SS_ERR_ARG, SS_ERR_DEVICE. */
ss_status ss_get_field(ss_grid g, int field, void* dst, int dst_on_device);

/* Advance every field by nsteps >= 0 semi-implicit spectral steps
 * (Eq. 8): per step the nonlinear terms of all fields are evaluated from
 * the current fields (Sec. 2.2.4, equation() before step()), transformed,
 * and combined with the transformed fields through A and B N_i.
 * Asynchronous on the grid's stream; it enqueues kernels only (no
 * memset, copy or synchronisation), so a caller may capture it into a HIP
 * graph on that stream and replay the graph, each replay taking the same
 * steps with the same bits, provided the carried spectrum is current when
 * captured (a step taken since the last ss_set_field), the captured step
 * count is even (the tuned arrangement may swap two arrays each step) and
 * no mass log is bound (its row index is fixed in the graph).
 * Errors: SS_ERR_STATE (model, workspace or a field missing), SS_ERR_ARG,
 * SS_ERR_DEVICE. */
ss_status ss_step_n(ss_grid g, int64_t nsteps);

/* ---- Stepping without allocation ----
 *
 * For callers that cannot allocate device memory or bind a workspace at
 * the point of the call: code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation.
 *
 * ss_step_fields_noalloc(g, fields, nsteps) does what ss_set_field (device
 * source) for every field, ss_step_n(g, nsteps) and ss_get_field (device
 * destination) for every field do, with the same arithmetic and results,
 * but keeps the spectral state and its spectrum in a fixed device array of
 * the library (SS_NOALLOC_SCRATCH_BYTES = 64 MiB per GPU, held from the
 * first use on that GPU until the process ends) instead of the grid's
 * workspace, and calls no allocating routine.
 *   fields[f]: device pointer to field f (0 .. nfields-1), a (nz, ny, nx)
 *     array of the grid dtype, read as the initial state and overwritten
 *     with the state after nsteps.  Caller-owned.
 *   Needs a model (ss_set_model / ss_set_equations), not a workspace; the
 *   grid's own workspace and fields are left untouched.  Steps are logged
 *   in the bound mass log like ss_step_n's.  Spectral solver only.
 *   Asynchronous on the grid's stream, which must belong to the current
 *   device.  Every call on one GPU uses the same array, which keeps the
 *   last call's contents: calls that overlap on one GPU (other streams,
 *   other threads) race and must be ordered by the caller.
 * ss_noalloc_scratch_bytes: *need = bytes this grid needs in the array
 *   (2 nfields arrays of 256-byte-aligned field size; with two explicit
 *   channels per field (ss_set_equations) nfields more in 2D, 2 nfields
 *   more in 3D), *limit = its size.
 * Errors: SS_ERR_ARG (null, nsteps < 0, need > limit, stream on another
 * device), SS_ERR_STATE (no model), SS_ERR_UNSUPPORTED (finite-difference
 * solver), SS_ERR_DEVICE. */
#define SS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
ss_status ss_step_fields_noalloc(ss_grid g, void* const fields[], int64_t nsteps);
ss_status ss_noalloc_scratch_bytes(ss_grid g, size_t* need, size_t* limit);

/* Optional finite check of the fields (failure detection): scans the
 * stored state of every field (the spectral state, where a NaN or an
 * infinity of any cell reaches every mode of its row, or the real fields
 * of the finite-difference solver) on the grid's stream and synchronises.
 * *nonfinite_fields = bit f set when field f holds a NaN or an infinity.
 * Returns SS_ERR_NONFINITE when any bit is set, SS_OK otherwise.  Uses
 * the first bytes of the grid's staging array.  Not called by ss_step_n,
 * which stays asynchronous: callers check between runs of steps.
 * Errors: SS_ERR_ARG (null), SS_ERR_STATE (no model, workspace or field),
 * SS_ERR_DEVICE. */
ss_status ss_check_finite(ss_grid g, int* nonfinite_fields);

/* Same as ss_step_n, and times every kernel launch with HIP events
 * recorded on the grid's stream between consecutive launches.  On return
 * (the stream is synchronised) pass_ms[i] holds the summed milliseconds of
 * pass kind i and pass_count[i] the number of launches, for i <
 * min(npass, SS_NPASS): 0 = x pass, 1 = k-space pass, 2 = inverse y pass,
 * 3 = forward y pass (3D only).  For measurement; ss_step_n is the
 * production entry point.
 * Errors: as ss_step_n, plus SS_ERR_ARG for null outputs. */
#define SS_NPASS 4
ss_status ss_step_n_profiled(ss_grid g, int64_t nsteps, double* pass_ms, int64_t* pass_count,
                             int npass);

/* Mean duration in milliseconds of one launch of pass kind `pass` (as in
 * ss_step_n_profiled) with the current tiling, from `nlaunch` back-to-back
 * launches between two events on the grid's stream (after one warm-up
 * launch).  While no field is stored (after binding the workspace, before
 * ss_set_field) every pass runs on the step's own arrays, so it moves the
 * traffic a step moves; the workspace contents are then undefined.  Once a
 * field is stored the launches leave the fields untouched: the x pass
 * reads the state and writes the scratch arrays, the k-space and y passes
 * run in place on the scratch and staging arrays (fewer distinct arrays
 * than a step: where a step's arrays outgrow the 256 MB Infinity Cache
 * these read faster than in a step).  For measurement.  Synchronises. */
ss_status ss_time_pass(ss_grid g, int pass, int nlaunch, double* mean_ms);

/* Choose the work decomposition of every kernel of the step for this
 * grid by timing each valid tiling (rows or lines per workgroup) `reps`
 * times on the grid's stream and keeping the fastest.  The tilings do not
 * change any result (each line is transformed by the same code whatever
 * its workgroup).  The choice is also remembered for later grids of the
 * same shape, dtype and model field count.  Timing as ss_time_pass: while
 * no field is stored the passes run on the step's own arrays (best called
 * then), layouts and the dominant tilings are compared by timing whole
 * steps, and so is whether a step's passes run in place on the state
 * arrays or write the nonlinear term to the scratch arrays (results are
 * bitwise the same); afterwards only the scratch and staging parts of the
 * workspace are written and the fields are untouched.
 * Synchronises the stream.  Errors: SS_ERR_STATE (no model/workspace),
 * SS_ERR_ARG (reps outside [1, 1000]), SS_ERR_DEVICE. */
ss_status ss_autotune(ss_grid g, int reps);

/* Read / override the tiling: tiles[0] = rows per x-pass workgroup (step),
 * tiles[1] = lines per k-space workgroup, tiles[2] = lines per y-pass
 * workgroup (3D), tiles[3] = rows per x-pass workgroup for set/get field,
 * tiles[4] = x-pass tiles per workgroup (0 or 1: one tile each; > 1: a
 * persistent x pass whose workgroups prefetch their next tile while
 * transforming the current one), tiles[5] = row block B of the spectral
 * layout (power of two; B consecutive rows of every kx are stored together,
 * B = ny*nz being the plain transposed layout).  In ss_set_tiles a 0 entry
 * keeps the current value; an invalid entry is SS_ERR_ARG; changing B
 * after a field was set is SS_ERR_STATE.  ss_autotune also chooses B when
 * no field is set yet. */
ss_status ss_get_tiles(ss_grid g, int tiles[6]);
ss_status ss_set_tiles(ss_grid g, const int tiles[6]);

/* Read / override which arrays a (stepping-form) step uses, chosen by
 * ss_autotune: 1 (default) every pass in place on the state arrays (the
 * k-space pass writes the new state over the nonlinear term), 0 the
 * nonlinear term in the scratch arrays and the new state back to the
 * state arrays, 2 the nonlinear term in the scratch arrays with the new
 * state written over it, after which the two arrays swap roles.  Results
 * are bitwise the same; only the memory traffic pattern differs.  A value
 * set here stays until changed here or by ss_autotune (tilings remembered
 * for the grid's shape do not replace it).
 * Errors: SS_ERR_ARG (null, arrangement outside 0..2). */
ss_status ss_get_step_arrangement(ss_grid g, int* arr);
ss_status ss_set_step_arrangement(ss_grid g, int arr);

/* ---- Reverse mode (adjoint) of ss_step_n ---------------------------------
 *
 * Gradients of a scalar J(q^T) of the fields after nsteps steps with
 * respect to the initial fields and the model coefficients, by the exact
 * transpose of the discrete step (the paper has no adjoint; the forward
 * map is the scheme of Sec. 2.4.2, Eqs. 3-4 and 8).  Implemented for 2D
 * Gray-Scott grids with axes up to 1024.  Memory: the fields are stored
 * every K steps during the forward run; the backward sweep recomputes one
 * segment of K steps at a time from its checkpoint.
 *
 * Sequence: ss_bind_adjoint_workspace(nsteps, K) -> set fields ->
 * ss_step_n_checkpointed (the fields advance to q^T) -> ss_adjoint_n. */
ss_status ss_adjoint_workspace_size(ss_grid g, int64_t nsteps, int K, size_t* bytes);
ss_status ss_bind_adjoint_workspace(ss_grid g, void* device_ptr, size_t bytes, int64_t nsteps, int K);

/* Advance nsteps (the scheme of ss_step_n, in the form that re-forms the
 * state's spectrum from the stored state every step, as the backward
 * sweep's recomputation does; the results agree with ss_step_n to
 * rounding) storing checkpoints every K steps. */
ss_status ss_step_n_checkpointed(ss_grid g);

/* Backward sweep.  dJ_dqT[f]: device (ny, nx) arrays of dJ/dq_f at the
 * final step (grid dtype).  dJ_dq0[f]: device outputs, dJ/dq_f at step 0.
 * dJ_dcoef: host double[4] receiving dJ/d(Du, Dv, F, k).  Synchronises
 * the stream.  Errors: SS_ERR_STATE (no checkpointed forward run, or the
 * coefficients or dt changed since), SS_ERR_ARG, SS_ERR_DEVICE. */
ss_status ss_adjoint_n(ss_grid g, const void* const dJ_dqT[], void* const dJ_dq0[], double* dJ_dcoef);

/* ---- Batched step: many independent grids in grouped launches ----------
 *
 * A batch advances several independent simulations together, the way the
 * paper's driver runs a list of models from one configuration one after
 * another (Sec. 2.4, Fig. 2), but with every member's tiles in the same
 * kernel launches: per step one grouped x-pass launch and one grouped
 * k-space launch cover all members, whatever their sizes and
 * coefficients.  A run of n steps can be captured into one HIP graph and
 * replayed with a single launch.
 *
 * Members: 2D grids of one dtype, single-field models (Allen-Cahn,
 * Cahn-Hilliard, PFC), nx and ny powers of two in [64, 2048], all
 * sharing the batch's stream, each with model, workspace and field set.
 * Results are bitwise those of ss_step_n on each member.  The mass log is
 * not written by batched steps.  Members must stay alive and keep their
 * workspaces while the batch exists. */
typedef struct ss_batch_s* ss_batch;

/* Create a batch over count >= 1 grids (copied handle list); the stream is
 * that of the first grid.  Members are stepped in parallel, so no two may
 * share workspace memory (a grid listed twice included).  Errors:
 * SS_ERR_ARG (null, mixed dtype or stream, shared workspace memory),
 * SS_ERR_UNSUPPORTED (3D, two-field model, size), SS_ERR_STATE (member
 * without model or workspace). */
ss_status ss_batch_create(const ss_grid* grids, int count, ss_batch* out);

/* Device bytes the batch needs for its member tables and the counters of
 * its single launches (caller-owned, 256-byte aligned, bound with
 * ss_batch_bind_workspace, which clears the counters and the error flag
 * on the batch's stream). */
ss_status ss_batch_workspace_size(ss_batch b, size_t* bytes);
ss_status ss_batch_bind_workspace(ss_batch b, void* device_ptr, size_t bytes);

/* Time each valid block size (128, 256, 512 threads) for the grouped
 * launches `reps` times and keep the fastest; then, unless ss_batch_set_mode
 * fixed the form, time 8 steps in each of the three forms below and keep
 * the fastest.  Fields are untouched (the timed
 * launches run on the members' scratch arrays).  Synchronises the stream. */
ss_status ss_batch_autotune(ss_batch b, int reps);

/* Form of the batched steps.  mode 0: grouped, two launches per step (x
 * pass, k-space pass), each covering the tiles of every member, the kernel
 * boundary ordering the passes.  mode 1: one launch for all the steps of a
 * call: each workgroup, as it starts, draws one work item (a tile of one
 * pass of one member at one step) from a ticket counter in (step, pass)
 * order, and per-member counters of finished tiles order the passes of
 * each member (its k-space tiles wait for its x tiles of the step, its next
 * x tiles for its k-space tiles), so the members advance independently
 * and the step boundary drains no launch; a small kernel resets the
 * counters before each launch.  mode 2: one cooperative launch for all
 * the steps of a call (as many workgroups as are resident at once, at most
 * one per tile of the larger pass): in each step workgroup g takes the
 * tiles g, g + G, ... of the x pass, waits at a device-wide barrier for
 * every workgroup, takes its k-space tiles the same way and waits again,
 * so that two barriers replace the two launches of a step (for a few small
 * grids, whose grouped steps are mostly launch gaps).  ss_batch_capture in
 * mode 2 records no graph: ss_batch_launch issues the cooperative launch
 * itself.  All forms run the same tile code and give the same bits.  Modes
 * 1 and 2 need one block size for both passes (SS_ERR_UNSUPPORTED
 * otherwise).  Waits inside the launches are bounded: one that runs out
 * makes every workgroup leave and is reported by ss_batch_check.
 * ss_batch_get_mode returns the current form (set here or by the tuner). */
ss_status ss_batch_set_mode(ss_batch b, int mode);
ss_status ss_batch_get_mode(ss_batch b, int* mode);

/* Synchronise the batch's stream; SS_ERR_DEVICE if a single launch gave
 * up a wait (its results are then incomplete). */
ss_status ss_batch_check(ss_batch b);

/* Bound of each wait of the single launch, in sleeps of about 128 cycles
 * (default 2^22, a fraction of a second; 0 gives up at the first unmet
 * wait, which tests of the failure path use). */
ss_status ss_batch_set_wait_limit(ss_batch b, unsigned limit);

/* Advance every member by nsteps on the stream (mode 0: 2 nsteps grouped
 * launches; mode 1: one launch). */
ss_status ss_batch_step_n(ss_batch b, int64_t nsteps);

/* Capture nsteps batched steps into a HIP graph (replaces a previous
 * capture): 2 nsteps grouped launches, or, in mode 1, the counter reset and
 * one launch.  The batch's stream must not be the null stream. */
ss_status ss_batch_capture(ss_batch b, int64_t nsteps);

/* Replay the captured graph once on the batch's stream (nsteps steps). */
ss_status ss_batch_launch(ss_batch b);

/* info[0] = threads per block of the grouped k-space launch (the grouped
 * x launch uses the largest power of two <= info[0] that tiles every
 * member), info[1], info[2] = blocks of the grouped x and k launches. */
ss_status ss_batch_info(ss_batch b, int info[3]);

/* Wait for the batch's stream (a captured run may still be executing),
 * then free the handle and its graph (not the caller's memory or the
 * member grids).  NULL is a no-op. */
ss_status ss_batch_destroy(ss_batch b);

/* Bind a device buffer of capacity * nfields doubles for the per-step
 * mass log (spatial mean of each field after each step; conserved for
 * Cahn-Hilliard and PFC, Sec. 3).  Entry (i, f) is at [i*nfields + f]
 * for the i-th step since the log was bound; steps beyond capacity are
 * not logged.  device_ptr = NULL unbinds. */
ss_status ss_bind_mass_log(ss_grid g, double* device_ptr, int64_t capacity);

/* Number of steps taken since the mass log was bound. */
ss_status ss_mass_log_count(ss_grid g, int64_t* count);

/* The logged rows copied to host memory: min(max, steps logged) rows of
 * nfields doubles (row i = step i since the log was bound), after the
 * grid's stream has finished the steps enqueued so far (synchronises the
 * stream).  *rows (may be NULL) receives the number copied.  dst_host is
 * only written during the call.  Errors: SS_ERR_ARG (null grid, negative
 * max, null dst_host with max > 0), SS_ERR_STATE (no log bound),
 * SS_ERR_DEVICE. */
ss_status ss_mass_log(ss_grid g, double* dst_host, int64_t max, int64_t* rows);

/* ---- Structure factor (Sec. 3, coarsening check against Porod's law) ----
 *
 * The radially averaged static structure factor of one field: the
 * occupancy rho = 1 where psi > 0 and 0 elsewhere (the positive phase
 * stands for the solid), its unnormalised DFT rho_hat over every axis,
 * S(k) = |rho_hat_k|^2 / N (N = cells, so that S summed over all modes is
 * the number of occupied cells), and the mean of S over the modes of each
 * radial bin b = round(|m|), m the integer mode vector (m_j in
 * -N_j/2 .. N_j/2 - 1).  Porod's law (Eq. 14) predicts S ~ k^-(d+1) in the
 * scaling regime; the paper averages S over 10 independent runs.
 *
 * ss_structure_factor_nbins: *nbins = number of bins of this grid,
 *   round(|m|max) + 1 with |m|max^2 = sum_j (N_j/2)^2.
 * ss_structure_factor: s_out[b] = mean S over bin b (0 for an empty bin),
 *   n_out[b] = number of modes in bin b; both device pointers of exactly
 *   nbins elements, written on the grid's stream (no synchronisation).
 *   The field's state is not modified; the grid's nonlinear-term scratch
 *   and staging arrays are overwritten (calls on one grid are ordered on
 *   its stream).  Within a workgroup the per-bin sums are kept in fixed
 *   point (2^-85 per term, exact integer adds), across workgroups they are
 *   added in a fixed order: a call gives the same bits every time for the
 *   grid's tiling.  Errors: SS_ERR_ARG (null pointer, field out of
 *   range, nbins not the grid's), SS_ERR_STATE (no model, workspace or
 *   field), SS_ERR_UNSUPPORTED (box lengths N_j dx_j not all equal, or no
 *   tiling fits). */
ss_status ss_structure_factor_nbins(ss_grid g, int* nbins);
ss_status ss_structure_factor(ss_grid g, int field, double* s_out, int64_t* n_out, int nbins);

/* Change the stream later calls enqueue on.  Work enqueued earlier on the
 * old stream is not waited for: the caller orders the two streams. */
ss_status ss_set_stream(ss_grid g, void* stream);

/* Free the handle (not the caller's device memory).  Does not wait for
 * work enqueued on the grid's stream, which may still use the caller's
 * buffers.  NULL is a no-op. */
ss_status ss_destroy_grid(ss_grid g);

/* Message of the last failed call on this thread ("" if none). */
const char* ss_last_error(void);

/* Library version string. */
const char* ss_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SPECSTEP_H */
