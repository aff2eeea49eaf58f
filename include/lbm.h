/*
 * lbm.h - C ABI of the MI355X thermal lattice Boltzmann library (liblbm.so).
 *
 * The library runs the lattice Boltzmann update of Shim's on-lattice
 * higher-order thermal models (the 2D 33-velocity model of Table 2 and the 3D
 * 95-velocity model of Table 3, both of order m = 4, and the lower-order 3D
 * 19- and 15-velocity sets of order m = 2 that the paragraph after
 * Formula (10) says the same construction gives):
 *
 *     f_i(x + e_i, t + 1) = (1 - omega) f_i(x, t) + omega f_i^eq(x, t)
 *
 * on a periodic grid (the update rule of the method; lattice units, dx = dt = 1,
 * particle displacement e_i per step), with the Hermite equilibrium
 * f_i^eq = w_i rho P^(N)(v_i) of order N = m (the polynomial-equilibrium form
 * next to Formula (2); N >= m as the paragraph after Formula (5) requires:
 * N = 4 for the models of Tables 2 and 3, N = 2 for the lower-order sets),
 * and the per-cell moments rho, U, T of the Maxwellian.  Around the update it
 * provides initialisation from macroscopic fields, moment output, global
 * conservation sums, the fixed end planes of the shock-tube experiment,
 * two-buffer or in-place (AA pattern) streaming, checkpointed runs and
 * resuming from their checkpoints, HIP-graph replay of step loops, a
 * hand-written adjoint that gives gradients of a loss on the final density
 * with respect to the initial temperature field and omega, and a general
 * constructor of on-lattice models (Formulas (5)-(10)).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns an lbm_status; no C++ exception crosses the ABI.
 *    On error the call has no side effect on the context and
 *    lbm_last_error() describes the failure.
 *  - Grid: extents (nx, ny[, nz]), every axis periodic, N = nx*ny[*nz] cells,
 *    linear cell index x + nx*(y + ny*z) (x fastest).
 *  - Populations in the bound buffers, checkpoints and adjoint workspace:
 *    row-blocked, i.e. the Q populations of a group of g consecutive grid
 *    rows are contiguous and population-major inside the group, the g rows
 *    of one population adjacent (g = 2 in 3D when ny is even, else 1):
 *    population i of cell (x, y, z) is element
 *    ((z*ny/g + y/g)*Q*g + i*g + y%g)*rs + x, with the run stride rs = nx
 *    rounded up to a multiple of 32 when nx >= 32 (two-buffer streaming; with
 *    LBM_STREAM_AA the slot of a value alternates, see lbm_set_streaming).
 *    The layout is internal to the library (sizes from
 *    lbm_workspace_bytes).  In
 *    LBM_FP64 each element is the double f*_i.  In LBM_FP32_SHIFTED each
 *    element is the float g_i = f*_i - w_i*rho0.  lbm_set_populations and
 *    lbm_get_populations exchange float64 f* in the order [Q][N] (element
 *    i*N + c) instead.
 *  - Stored state: the post-collision populations
 *    f*_i(x, t) = (1 - omega) f_i(x, t) + omega f_i^eq(x, t), i.e. the
 *    right-hand side of the update rule; the next step moves them to x + e_i,
 *    f_i(x + e_i, t + 1) = f*_i(x, t).  Collision conserves rho, rho U and
 *    sum f |e|^2, so the moments of f* are those of f at time t.  After
 *    lbm_init_fields, f* = f = f^eq.
 *  - Macroscopic fields are float64 device arrays: rho[N], U[D][N]
 *    (component-major, components x, y[, z]), T[N].  U is in cells per step,
 *    T = k_B T / m_g in cells^2/step^2; the reference temperature is
 *    T0 = 1/(2 c^2) (the dimensionless variables v = Theta^(-1/2) V with
 *    Theta = 2 k_B T0 / m_g and v_i = c e_i).
 *  - Memory: the library allocates no device memory.  Population buffers,
 *    scratch, checkpoints, workspaces and fields are owned by the caller
 *    (e.g. torch tensors); the library never frees them.  Buffers given to
 *    lbm_bind must be 256-byte aligned, other device arrays 8-byte aligned;
 *    all must stay valid while the context uses them.
 *  - Asynchrony: kernels run on the stream given to lbm_create, in order.
 *    Functions that return host values (lbm_conservation, lbm_adjoint's
 *    omega gradient) synchronise that stream.
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum lbm_status {
    LBM_OK = 0,
    LBM_E_INVALID = -1,      /* bad argument: value, size, alignment, pointer */
    LBM_E_UNSUPPORTED = -2,  /* velocity set or precision the library has no kernel for */
    LBM_E_DEVICE = -3,       /* a HIP runtime call or kernel launch failed */
    LBM_E_STATE = -4,        /* call out of order (not bound / not initialised) */
    LBM_E_NONFINITE = -5     /* a reduced diagnostic is NaN or infinite */
} lbm_status;

typedef enum lbm_streaming {
    LBM_STREAM_AB = 0,       /* two population buffers, pull from one into the other (default) */
    LBM_STREAM_AA = 1        /* one buffer updated in place (AA pattern), half the memory */
} lbm_streaming;

typedef enum lbm_precision {
    LBM_FP64 = 0,            /* populations and arithmetic in float64 */
    LBM_FP32_SHIFTED = 1     /* float32 deviations g_i = f_i - w_i rho0, float32 arithmetic */
} lbm_precision;

/* Largest number of velocities of a supported model. */
#define LBM_MAX_Q 95

/*
 * lbm_velocity_set - the canonical velocity set of a supported model and its
 * weights, solved on the host.
 *
 * Builds the union of the symmetry groups of Table 2 (D = 2, Q = 33),
 * Table 3 (D = 3, Q = 95) or of a lower-order 3D set (Q = 19: the groups of
 * (0,0,0), (1,0,0), (1,1,0); Q = 15: (0,0,0), (1,0,0), (1,1,1)): each group
 * is the orbit of its representative under coordinate permutations and sign
 * changes (the group construction before Formula (9)).  Canonical order:
 * groups in that order, vectors of a group sorted ascending as integer
 * tuples.  Then solves the square system of Formula (5) (even moments up to
 * n_max = 2m: m = 4 for Tables 2 and 3, Omega(4, D) equations; m = 2 for the
 * lower-order sets, Omega(2, 3) = 4 equations; Formula (10) unknowns: one
 * weight per group plus c) by Newton's method in binary128, started from the
 * printed table values (the lower-order sets: least-squares weights at
 * c = 1), and rounds the root to float64.  The right-hand side is
 * normalised so that the weights sum to one.
 *
 *   D, Q  : 2 and 33, or 3 and 95, 19 or 15; otherwise LBM_E_UNSUPPORTED.
 *   e     : host int32[Q][D] out, displacements (may be NULL).
 *   w     : host double[Q] out, weight of each velocity (may be NULL).
 *   c     : host double out, the speed of Formula (5) (may be NULL).
 * Returns LBM_E_DEVICE never; LBM_E_INVALID if Newton fails to converge.
 */
int lbm_velocity_set(int D, int Q, int32_t* e, double* w, double* c);

/*
 * lbm_equation_count - Omega(m, D) of Formula (8): the number of equations
 * Formula (5) gives up to order 2m in D dimensions, one per partition of
 * q <= m into at most D parts (Table 1).  0 <= m <= 16, 1 <= D <= 8.
 */
int lbm_equation_count(int m, int D, int* count);

/*
 * lbm_model_build - construct an on-lattice model from a choice of groups
 * (the method of the counting section, Formulas (5) and (8)-(10)).
 *   D, m      : dimension (1, 2 or 3) and order of accuracy (1..8); the
 *               equations are Formula (5) for every even multi-index of
 *               order <= 2m.
 *   G, reps   : number of groups and host int32[G][D] representatives; each
 *               group is the orbit of its representative under coordinate
 *               permutations and sign changes (components in [-64, 64]).
 *               Formula (10) must hold: G + 1 = Omega(m, D).
 *   w_guess   : host double[G] initial group weights, or NULL for the least
 *               squares weights at c_guess; c_guess > 0 initial speed.
 *   q_cap     : rows available in e and group.
 * Outputs (any may be NULL): e int32[Q][D] in canonical order (groups in
 * the given order, ascending tuples inside a group), group int32[Q],
 * w double[Q] per velocity, c, Q, residual (largest |Formula (5) residual|
 * at the float64 result).  The square system is solved by Newton in
 * binary128 and rounded once; with the representatives and printed values
 * of Table 2 or 3 the result equals lbm_velocity_set bit for bit.
 * Returns LBM_E_UNSUPPORTED for other D, LBM_E_INVALID for a system that is
 * not square, repeated groups, no convergence, a non-positive weight or c,
 * or q_cap < Q (Q is still reported in the last case).  The sets with
 * kernels are those of lbm_velocity_set (lbm_create): built here from the
 * same representatives (and m = 2 for the lower-order 3D sets) they are
 * accepted by lbm_create.
 */
int lbm_model_build(int D, int m, int G, const int32_t* reps, const double* w_guess,
                    double c_guess, int q_cap, int32_t* e, int32_t* group, double* w, double* c,
                    int* Q, double* residual);

/*
 * lbm_create - validate a model and a grid and make a context.
 *
 *   out       : receives the context (host memory owned by the library,
 *               released by lbm_destroy).
 *   D, Q, e   : dimension, velocity count and host int32[Q][D]
 *               displacements; must equal a supported model in canonical
 *               order (see lbm_velocity_set: D2Q33, D3Q95, D3Q19, D3Q15),
 *               else LBM_E_UNSUPPORTED.
 *   w         : host double[Q] weights: positive, equal within each group,
 *               summing to 1 within 1e-12.
 *   c         : speed of the model; Formula (5) (up to n_max = 2m of the
 *               model) must hold at (w, c) with residual <= 1e-10, else
 *               LBM_E_INVALID.
 *   extent    : host int64[D] = {nx, ny[, nz]}, each >= 1 and <= 2^24,
 *               N < 2^31 cells (more than 288 GB of populations); the
 *               populations of one slab of the slowest axis (nx*ny*Q
 *               elements in 3D, nx*Q in 2D) must stay below 4 GiB.
 *   omega     : relaxation frequency of the update rule, 0 <= omega < 2.
 *               (omega = 0 turns the update into pure streaming.)
 *   precision : LBM_FP64 or LBM_FP32_SHIFTED.
 *   rho0      : shift reference density for LBM_FP32_SHIFTED (>= 0, finite;
 *               1 for flows with mean density one); ignored for LBM_FP64.
 *   stream    : hipStream_t on which every kernel of this context runs
 *               (NULL = the default stream).
 * No device call is made; the context is unbound until lbm_bind.
 */
int lbm_create(lbm_ctx** out, int D, int Q, const int32_t* e, const double* w,
               double c, const int64_t* extent, double omega, int precision,
               double rho0, void* stream);

/*
 * lbm_workspace_bytes - sizes of the caller-owned buffers for lbm_bind.
 *   pop_bytes     : bytes of one population buffer (Q * N * element size).
 *   scratch_bytes : bytes of the reduction scratch buffer.
 */
int lbm_workspace_bytes(const lbm_ctx* ctx, size_t* pop_bytes, size_t* scratch_bytes);

/*
 * lbm_set_streaming - choose how a step moves the populations; call before
 * lbm_bind (LBM_E_STATE after it).
 *   LBM_STREAM_AB (default): two buffers; a step gathers f*_i(x - e_i) from
 *     one and writes f*(t + 1) to the other.
 *   LBM_STREAM_AA: one buffer updated in place, so a grid twice as large fits
 *     in the same memory.  Steps alternate between a kernel that reads the
 *     arriving values from the neighbours' opposite slots and writes each
 *     result into the neighbour it streams to, and a kernel that reads and
 *     writes its own cell only (populations stored in the opposite slot).
 *     Every location is read and written by one thread only.  The update
 *     (the update rule that opens the method) and its arithmetic are those
 *     of LBM_STREAM_AB (bit-identical results);
 *     lbm_moments, lbm_conservation and lbm_get/set_populations follow the
 *     alternating storage, and held planes (lbm_set_fixed_planes) store
 *     f^eq of their state into the locations they own in either kernel, so
 *     they too give the LBM_STREAM_AB result bit for bit.
 *     lbm_run_checkpointed copies its snapshots out of the buffer in the
 *     LBM_STREAM_AB layout, so lbm_adjoint works with either scheme and
 *     gives the same gradients bit for bit.
 * Returns LBM_E_INVALID for another scheme.
 */
int lbm_set_streaming(lbm_ctx* ctx, int scheme);

/*
 * lbm_bind - attach caller-owned device memory: population buffers f_a and
 * f_b (LBM_STREAM_AB: both, distinct; LBM_STREAM_AA: f_a only, f_b must be
 * NULL) and a scratch buffer, of the sizes lbm_workspace_bytes reports, all
 * 256-byte aligned.  Records the current HIP device.  Re-binding is allowed
 * and drops the initialised state.
 */
int lbm_bind(lbm_ctx* ctx, void* f_a, void* f_b, void* scratch);

/*
 * lbm_init_fields - set the populations to the equilibrium of the given
 * fields, f_i = f_i^eq(rho, U, T) at every cell (the homogeneous initial
 * states of the shock-tube experiment are given this way).  Computed in
 * float64 and, for LBM_FP32_SHIFTED, rounded once to float.
 *   rho[N], U[D][N], T[N] : device float64 inputs; rho > 0 and T > 0 are
 *   the caller's responsibility (not checked).
 */
int lbm_init_fields(lbm_ctx* ctx, const double* rho, const double* U, const double* T);

/*
 * lbm_set_populations / lbm_get_populations - copy the stored state f* (see
 * above) from / to a device float64 array f[Q][N] holding f*_i (not the
 * shifted value).  For LBM_FP32_SHIFTED the setter stores
 * float(f*_i - w_i rho0).
 */
int lbm_set_populations(lbm_ctx* ctx, const double* f);
int lbm_get_populations(lbm_ctx* ctx, double* f);

/*
 * lbm_step - advance n >= 0 time steps of the update rule.  Each step is one
 * kernel: gather f_i(x, t + 1) = f*_i(x - e_i, t) (periodic, any extent),
 * moments, 4th-order equilibrium, BGK relaxation, coalesced store of
 * f*(x, t + 1).  Asynchronous.
 */
int lbm_step(lbm_ctx* ctx, int n);

/*
 * lbm_tune_step - lbm_step(ctx, n), timing on the way the order in which
 * the forward steps hand out their blocks, and keeping the faster order for
 * the steps that follow.
 *
 * The blocks of a forward step (two-buffer or in place) are dispatched
 * round-robin over the 8 XCDs of the device.  Order 0 (the default) gives each XCD a contiguous
 * range of rows; order 1 gives the XCDs one slab of the slowest axis (a
 * z-plane in 3D, a row in 2D) in turn.  Which is faster depends on where in
 * HBM the bound buffers lie (measured on D3Q95 FP32-shifted 384^3: order 1
 * 0.4-1.3 % faster on some placements, 1.5-2 % slower on others; in place
 * 0.5 % faster on the placements measured).  The
 * order only decides which blocks run where: every step, the checkpointed
 * forward run and the recomputation in lbm_adjoint give bit-identical
 * results under both, and the kernels that sum across blocks (conservation,
 * adjoint) keep order 0, so their rounding does not depend on it.
 *
 *   n       : steps to run (>= 0); the result equals lbm_step(ctx, n) bit
 *             for bit.  The steps alternate the two orders (in place: per
 *             pair of steps, one of each kernel), each step between two
 *             events on the context's stream; the first step (pair) of each
 *             order counts as warm-up when n >= 6 (in place 12).
 *   mapping : host int out (may be NULL), the order kept: 0 or 1.
 * Tuning needs n >= 4 (in place 8) and a stream that is not being captured;
 * otherwise this is lbm_step(ctx, n) and the order stays.  The
 * call synchronises the stream when it tunes.  lbm_bind resets the order
 * to 0.  Errors as lbm_step.
 */
int lbm_tune_step(lbm_ctx* ctx, int n, int* mapping);

/*
 * lbm_set_block_order - set the forward steps' block order of lbm_tune_step
 * directly (0 or 1, else LBM_E_INVALID), e.g. to repeat a tuned choice or to
 * compare the two.  No device call; results do not depend on it.
 */
int lbm_set_block_order(lbm_ctx* ctx, int order);

/*
 * lbm_moments - rho, U, T of the current populations (Formula (1) with
 * n = 0, 1, 2): rho = sum f_i, U = sum f_i e_i / rho,
 * T = (sum f_i |e_i|^2 / rho - |U|^2) / D.  Outputs are device float64
 * arrays rho[N], U[D][N], T[N] (any of them may be NULL).  Asynchronous.
 */
int lbm_moments(lbm_ctx* ctx, double* rho, double* U, double* T);

/*
 * lbm_conservation - global sums of the conserved quantities of the current
 * populations, reduced in float64 in a fixed order (bitwise repeatable):
 *   out[0] = mass sum_x sum_i f_i, out[1..D] = momentum sum_x sum_i f_i e_i,
 *   out[D+1] = energy sum_x sum_i f_i |e_i|^2 / 2.
 *   out : host double[D+2].  Synchronises the stream.
 * Returns LBM_E_NONFINITE (and still fills out) if any sum is not finite.
 */
int lbm_conservation(lbm_ctx* ctx, double* out);

/*
 * lbm_conservation_noalloc - lbm_conservation for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same kernels and the same sums, bit
 * for bit, but the reduction partials and the reduced values live in a static
 * device array of the library (41.5 KB, one per GPU, kept until the process
 * ends) instead of the scratch buffer given to lbm_bind.  No device memory is
 * allocated or freed; the first call on a GPU looks up that GPU's array.
 * Every grid the library accepts fits (at most 1024 partials of D + 2
 * values); a grid that needed more would be refused with LBM_E_INVALID.
 * Calls on one GPU share the array: calls that overlap in time on one GPU
 * (from several host threads, or on several streams before the previous
 * call returned) race; each call overwrites every element it reads, so
 * consecutive calls need no clearing.  Synchronises the stream, like
 * lbm_conservation.
 */
int lbm_conservation_noalloc(lbm_ctx* ctx, double* out);

/*
 * lbm_stream_copy - measurement reference, not part of the method: copies the
 * current populations (LBM_STREAM_AB) into the other bound buffer n times
 * with a plain streaming kernel (one 16-byte vector per lane, non-temporal
 * stores), i.e. the bytes of one update step (each population read once and
 * written once) without its gather and arithmetic, on the same buffers: the
 * read + write rate HBM sustains for this state, against which the step's
 * rate is compared.  The state is not changed (the other buffer is the next
 * step's destination anyway).  Asynchronous.  LBM_E_STATE before
 * lbm_init_fields, LBM_E_UNSUPPORTED with LBM_STREAM_AA (one buffer),
 * LBM_E_INVALID for n < 0.
 */
int lbm_stream_copy(lbm_ctx* ctx, int n);

/*
 * lbm_set_fixed_planes - the shock-tube end conditions of the experiment in
 * the results section: the first n_lo and the last n_hi planes along the
 * slowest axis (the XY-planes at the two ends of z in 3D, the X-rows at the
 * two ends of y in 2D) are held at the equilibrium f^eq(state) of a fixed
 * macroscopic state; the other axes stay periodic.
 *   state_lo, state_hi : host double[D+2] = {rho, U_x, U_y[, U_z], T}
 *                        (rho > 0, T > 0, finite); read during the call
 *                        and copied; may be NULL where the count is 0.
 * After every subsequent update step of lbm_step the held planes are
 * overwritten with f^eq(state), which the collision leaves unchanged, so
 * they act as reservoirs.  The populations a cell gathers come from at most
 * max|e_z| planes away (5 for D3Q95, 4 for D2Q33 along y): with
 * n_lo, n_hi >= that, no interior cell gathers across the periodic seam.
 * The held planes are not touched until the next step (set the initial
 * state with lbm_init_fields).  n_lo = n_hi = 0 restores a fully periodic
 * lattice.  Returns LBM_E_INVALID for n_lo, n_hi < 0, n_lo + n_hi >
 * extent[D-1], NULL or non-positive states, LBM_E_NONFINITE for NaN/Inf.
 * Works with both streaming schemes.
 * lbm_run_checkpointed works with held planes, and so does the temperature
 * gradient of lbm_adjoint (see there); its omega gradient needs an
 * all-periodic lattice.
 */
int lbm_set_fixed_planes(lbm_ctx* ctx, int n_lo, int n_hi, const double* state_lo,
                         const double* state_hi);

/*
 * lbm_set_graph_steps - replay lbm_step in HIP graphs of `steps` update steps
 * (the update rule, unchanged): the first call that needs them captures the
 * launches of `steps` steps once, later calls replay the graph for every full
 * block of `steps` steps and launch the remainder one by one.  Launch-bound
 * small grids (the shock tube) gain; the arithmetic and results are the same
 * bit for bit.  steps must be even (the buffers and storage form return to
 * their state after an even count), 0 turns replay off (the default).  The
 * graph is rebuilt after lbm_bind, lbm_set_omega or lbm_set_fixed_planes.
 * Needs a non-null stream (LBM_E_UNSUPPORTED otherwise); LBM_E_INVALID for
 * odd or negative steps.  Graphs hold no memset nodes.
 */
int lbm_set_graph_steps(lbm_ctx* ctx, int steps);

/* lbm_set_omega - change the relaxation frequency (0 <= omega < 2). */
int lbm_set_omega(lbm_ctx* ctx, double omega);

/*
 * lbm_checkpoint_bytes - size of the checkpoint buffer of an n-step run with
 * a snapshot every k steps whose last `keep` segments keep the moments of
 * their steps: ceil(n/k) + 1 population buffers (256-byte aligned slots) plus
 * D+2 moment planes in storage precision for each step of those segments.
 * keep >= 1; keep >= ceil(n/k) keeps the moments of every step (the adjoint
 * then recomputes nothing; 20 B per cell per step in LBM_FP32_SHIFTED).
 */
int lbm_checkpoint_bytes(const lbm_ctx* ctx, int n, int k, int keep, size_t* bytes);

/*
 * lbm_run_checkpointed - like lbm_step(n), and fills ckpt for lbm_adjoint:
 * the stored state at t = 0, k, 2k, ... (before the step that starts each
 * segment) in slot s = t/k, the final state in slot ceil(n/k), and after the
 * slots the moments of every step of the last `keep` segments.  Snapshot 0
 * is a copy of the bound state; later snapshots are written in place by the
 * step that produces them (LBM_STREAM_AA: every snapshot and the final state
 * are copied out of the in-place buffer in the two-buffer layout).
 * n >= 1, k >= 1, keep >= 1.
 */
int lbm_run_checkpointed(lbm_ctx* ctx, int n, int k, int keep, void* ckpt, size_t ckpt_bytes);

/*
 * lbm_restore_checkpoint - resume a run from a checkpoint buffer filled by
 * lbm_run_checkpointed(n, k, keep) of a context with the same model, grid,
 * precision and rho0 (checkpoint/resume; the state is the one the update
 * rule advances).
 *   slot : 0 .. ceil(n/k) - 1 restores the stored state at t = slot*k;
 *          ceil(n/k) restores the final state at t = n.
 * The snapshot is copied into the bound populations (in place: into the
 * in-place form), so lbm_step(m) then continues exactly as the original run
 * did, bit for bit, with the context's current omega.  Asynchronous on the
 * stream; the buffer must stay valid until the copy has run.
 * LBM_E_STATE before lbm_bind; LBM_E_INVALID for n, k, keep < 1, a slot out
 * of range or a buffer smaller than lbm_checkpoint_bytes(n, k, keep).
 */
int lbm_restore_checkpoint(lbm_ctx* ctx, int n, int k, int keep, const void* ckpt,
                           size_t ckpt_bytes, int slot);

/*
 * lbm_adjoint_workspace_bytes - size of the workspace lbm_adjoint needs for
 * the same (n, k, keep): three population-sized buffers (adjoint ping-pong
 * and recomputation), k steps of stored moments when some segment is
 * recomputed, the float64 reduction partials and one float64 per segment.
 */
int lbm_adjoint_workspace_bytes(const lbm_ctx* ctx, int n, int k, int keep, size_t* bytes);

/*
 * lbm_adjoint - gradient of a loss L(rho_n) of the density after n steps
 * with respect to the initial temperature field and omega.
 *
 * The forward map is f*^0 = f^eq(rho_init, U_init, T_init), then n updates
 * f*^{t+1} = C(S f*^t) with S the streaming and C the collision at the
 * moments m^{t+1} of S f*^t.  The adjoint runs backwards over the segments of
 * a checkpointed run (lbm_run_checkpointed with the same n, k, keep, from the
 * same initial fields): for each segment whose moments were not kept it
 * recomputes the forward steps from the checkpoint, storing the D+2 moments
 * of each step, then applies
 *   nu^t_i(x) = (1 - omega) mu_i + omega (G_rho + G_j . e_i + G_E |e_i|^2),
 *   mu_i = nu^{t+1}_i(x + e_i),  G_m = sum_k mu_k d f_k^eq / d m at m^t,
 * with m = (rho, rho U, sum f |e|^2), for t = n-1 .. 1, from
 * nu^n_i(x) = dL/drho_n(x); dL/df*^0 is the transposed streaming of nu^1.
 * Because the update is homogeneous of degree one in f, K(t) = <nu^t, S f*^{t-1}>
 * is the same for every t (K(n) = sum_x dL/drho_n rho_n), so
 *   dL/domega = sum_{t=1}^{n-1} (sum_x sum_i mu_i f_i^eq(m^t) - K(t+1)) / (1 - omega)
 * needs only the stored moments; it is reduced in float64.  The adjoint
 * state is stored (and rounded) in the storage precision, which makes K
 * drift slowly; K is therefore measured at t = s k + 1 against each snapshot
 * and at t = n, and K(t) is taken linearly between those points.
 *
 *   ckpt, ckpt_bytes   : the checkpoints of the forward run.
 *   rho_init, U_init, T_init : device float64 initial fields of that run.
 *   dL_drho_final      : device float64[N], dL/drho_n.
 *   workspace, ws_bytes: device buffer of lbm_adjoint_workspace_bytes(n, k, keep).
 *   dL_dT_init         : device float64[N] out (may be NULL).
 *   dL_domega          : host double out (may be NULL); when requested,
 *                        |1 - omega| >= 1e-3 is required (LBM_E_INVALID
 *                        otherwise) and the call synchronises the stream.
 *                        Accuracy: A - K nearly cancels and is divided by
 *                        1 - omega, so the LBM_FP32_SHIFTED error grows like
 *                        1/|1 - omega| (measured against central differences
 *                        of the float64 run, D3Q95 48x40x32, 60 steps, over
 *                        several runs: 3.4e-5 to 1.0e-4 at omega = 0.9,
 *                        2.2e-4 to 4.4e-4 at omega = 1.05; 128^3, 200 steps:
 *                        5e-6 to 7e-6 at omega = 1.4).  LBM_FP64 stays near
 *                        1e-12 relative.
 * With held planes (lbm_set_fixed_planes, set as in the forward run) the
 * post-collision values of held cells are constants: their adjoint state is
 * zero at every t <= n, and the initial field on the held planes still
 * counts through the first step.  The omega gradient, which relies on the
 * homogeneity of the all-periodic step, is then refused (LBM_E_UNSUPPORTED);
 * request dL_dT_init alone.
 * The context's populations are left as they were.
 */
int lbm_adjoint(lbm_ctx* ctx, int n, int k, int keep, const void* ckpt, size_t ckpt_bytes,
                const double* rho_init, const double* U_init, const double* T_init,
                const double* dL_drho_final, void* workspace, size_t ws_bytes,
                double* dL_dT_init, double* dL_domega);

/* lbm_destroy - release the context (not the caller's device memory). */
int lbm_destroy(lbm_ctx* ctx);

/* Static description of a status code. */
const char* lbm_status_str(int status);

/* Detail of the last failure of this context ("" if none).  With ctx == NULL,
 * the last failure of lbm_create / lbm_velocity_set on this thread. */
const char* lbm_last_error(const lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
