/*
 * tgexp -- split exponential Euler for diffusion-reaction systems on the
 * disk, sphere, ball and cylinder, on AMD Instinct MI355X (gfx950).
 *
 * The method is that of Caliari & Cassini, "A tensor-based exponential
 * integrator for diffusion-reaction equations in common curvilinear
 * coordinates":
 *   - grids and 1D finite-difference operators: Section 3, Table 1,
 *     eqs. (A_theta), (disk_discr), (ball_discr), (syscn), (A_phi), (A_z);
 *   - Kronecker-sum Laplacians M = M_1 + ... + M_d: Section 2,
 *     eqs. (disk), (sphere), (ball), (cylinder);
 *   - one step for species s of an N-coupled system (Section 4, eqs.
 *     (ee), (splitorder), (BVAM_SExpE)):
 *         F_s   = d_s M W_s + g_s(W)
 *         W_s  <- W_s + tau phi_1(tau d_s M_1) ... phi_1(tau d_s M_d) F_s,
 *     the factors applied as mu-mode products in the order of eqs.
 *     (ee_disk), (ee_sphere), (ee_ball), (ee_cylinder) (M_d first).
 *
 * Conventions
 *   - Every function returns 0 (TG_OK) or a negative TG_E* code; the text
 *     of the last error of the calling thread is returned by
 *     tg_last_error().  Nothing throws across this interface.
 *   - Grid sizes n[] are given in the paper's coordinate order:
 *       disk (n_rho, n_theta); sphere (n_theta, n_phi);
 *       ball (n_rho, n_theta, n_phi); cylinder (n_rho, n_theta, n_z).
 *     Each n must be >= 3.
 *   - State layout (device memory, caller-owned): C-contiguous
 *     [batch][n_species][n3][n2][n1], first coordinate fastest, i.e. the
 *     paper's vectorisation w_{i + (j-1) n1 + (k-1) n1 n2} per species
 *     (2D: n3 = 1).  Element type is double for TG_FP64 and float for
 *     TG_FP32 / TG_BF16X2 / TG_BF16X3.
 *   - The state holds deviations W - w_ref from a per-(instance, species)
 *     reference state (by default the homogeneous equilibrium of the
 *     reaction).  For the cylinder the Dirichlet value at z_* is w_ref.
 *   - Device buffers (state, hook inputs and outputs) must be aligned to 4
 *     elements (16 bytes for float, 32 for double); TG_EINVAL otherwise.
 *   - Device pointers and the hipStream_t argument (passed as void*, NULL =
 *     default stream) are the caller's; calls enqueue work asynchronously
 *     unless stated otherwise.  A plan owns its device factors and scratch
 *     buffers until tg_plan_destroy.  Calls on one plan must not overlap.
 */
#ifndef TGEXP_H
#define TGEXP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  TG_OK = 0,
  TG_EINVAL = -1,     /* invalid argument (sizes, kinds, null pointers) */
  TG_ENOMEM = -2,     /* device or host allocation failed */
  TG_EHIP = -3,       /* HIP runtime error (launch, copy, graph) */
  TG_ENOTSUP = -4,    /* combination not supported */
  TG_ENONFINITE = -5  /* a non-finite value was produced by the update */
};

/* Geometries (Section 2, eqs. (disk)-(cylinder)); TG_DISK_LAMBDA is the
 * unit-radius-scaled disk with the anomalous operator Delta_lambda of
 * Section 5.3 (eqs. (anomalous), (A_lambda)): radial operator A_lambda with
 * Dirichlet data at rho_*, D_rho = rho^(-2-lambda), periodic theta. */
enum { TG_DISK = 0, TG_SPHERE = 1, TG_BALL = 2, TG_CYLINDER = 3, TG_DISK_LAMBDA = 4 };

/* Arithmetic of the mu-mode products.  Factors are always computed in
 * FP64 on the host and rounded to the storage type.
 *   TG_FP64   : FP64 MFMA, FP64 state.
 *   TG_FP32   : FP32 MFMA, FP32 state.
 *   TG_BF16X2 : FP32 state; each product operand carried as two bf16 terms
 *               (x ~ hi + lo), three bf16 MFMA products (hi.hi, hi.lo, lo.hi)
 *               accumulated in FP32 (representation error about 2^-17 relative per
 *               operand, so about 2^-16 per product).
 *   TG_BF16X3 : three bf16 terms, six products (about 2^-24 relative).
 * The split-bf16 precisions run on the fused routes only (0 and 2) and
 * tg_plan_create returns TG_ENOTSUP where those do not fit the grid. */
enum { TG_FP64 = 0, TG_FP32 = 1, TG_BF16X2 = 2, TG_BF16X3 = 3 };

/* Reaction g(w) (explicit, evaluated at t_n).  params per instance:
 *   TG_REACT_SCHNAKENBERG: (a, b):  g_u = a - u + u^2 v,  g_v = b - u^2 v
 *       (paper eq. (schnaknl) with alpha_1 = 1); equilibrium
 *       (a + b, b / (a + b)^2).
 *   TG_REACT_AIS3: (a, b, kappa, mu), three species (u, v, w):
 *       g_u = a - u + u^2 v - kappa u w, g_v = b - u^2 v, g_w = mu (u - w).
 *   TG_REACT_SCHNAKENBERG_SCALED: (a, b, gamma): gamma times the
 *       Schnakenberg terms (eqs. (schnaksys), (schnaknl): a = alpha_2,
 *       b = beta_1, gamma = alpha_1); same equilibrium.
 *   TG_REACT_LINEAR: (k_0, c_0, k_1, c_1, ...), up to three species:
 *       g_s = -k_s (w_s - c_s) (the bulk kinetics b, c of eq. (bulkcylnl),
 *       Section 5.6, with (alpha1, alpha2, beta1, beta2)); equilibrium c_s.
 *   TG_REACT_DIB: (zeta1, zeta2, zeta3, zeta4, zeta5, eta1, eta2, eta3,
 *       eta4, eta5), two species (r, s): g_r = zeta1 p, g_s = zeta1 q with
 *       p = zeta2 (1 - s) r - zeta3 r^3 - zeta4 (s - zeta5),
 *       q = eta1 (1 + eta2 r)(1 - s)(1 - eta3 (1 - s))
 *           - eta4 (1 + eta5 r) s (1 + eta3 s)
 *       (eqs. (DIB), Section 5.4; in the bulk-surface step of Section 5.6
 *       the factors u of p and v of q are the cylinder's values below the
 *       point, eq. (bulkcylnl)); reference (0, zeta5).
 *   TG_REACT_NONE: g = 0 (pure diffusion).
 * Plans with TG_REACT_LINEAR or TG_REACT_DIB compute F in a stencil launch
 * of their own (route 0 behaves as route 2, route 4 is not offered) and have
 * no adjoint (TG_ENOTSUP). */
enum {
  TG_REACT_NONE = 0,
  TG_REACT_SCHNAKENBERG = 1,
  TG_REACT_AIS3 = 2,
  TG_REACT_SCHNAKENBERG_SCALED = 3,
  TG_REACT_LINEAR = 4,
  TG_REACT_DIB = 5
};

/* tg_apply_operator selectors */
enum { TG_APPLY_F = 0, TG_APPLY_DIFFUSION = 1, TG_APPLY_REACTION = 2 };

typedef struct tg_grid_s* tg_grid;
typedef struct tg_plan_s* tg_plan;

/* Thread-local text of the last failure; never NULL. */
const char* tg_last_error(void);
/* Interface version (incremented on incompatible change). */
int tg_version(void);

/* ---- grid and operator set-up (host, FP64) ------------------------------
 * extent = {rho_*, z_*}: radius of disk / ball / cylinder, or of the sphere
 * (its operator is scaled by rho_*^-2), and the cylinder height (ignored
 * elsewhere).  NULL means {1, 1}.  Section 3, Table 1.  For TG_DISK_LAMBDA
 * extent = {rho_*, lambda} is required, with lambda < 1 (the first grid
 * point (1 - lambda) h / 2 must be positive). */
int tg_grid_create(int32_t geometry, const int32_t* n, const double* extent, tg_grid* out);
int tg_grid_destroy(tg_grid g);
/* ndim (2 or 3) and the n[] of the grid (n must hold 3 ints). */
int tg_grid_dims(tg_grid g, int32_t* ndim, int32_t* n);
/* Grid points of mode mode (1-based): rho_i, theta_j, phi_k or z_k. */
int tg_grid_coords(tg_grid g, int32_t mode, double* out);
/* The tridiagonal 1D operator of mode `mode` (unscaled, without D_rho /
 * D_phi): row r has lo[r] (column r-1), diag[r], up[r] (column r+1).  For
 * the periodic theta operator lo[0] couples to column n-1 and up[n-1] to
 * column 0; otherwise those two entries are 0. */
int tg_grid_operator(tg_grid g, int32_t mode, double* lo, double* diag, double* up);
/* Real eigen-decomposition A = V diag(lam) Vinv of mode `mode`'s operator
 * (row-major n x n; Proposition 1 for the tridiagonal ones, the closed-form
 * real Fourier basis for theta). */
int tg_grid_eig(tg_grid g, int32_t mode, double* lam, double* V, double* Vinv);
/* phi_1(c A) of mode `mode`'s operator, row-major n x n (Section 4). */
int tg_grid_phi1(tg_grid g, int32_t mode, double c, double* out);

/* ---- plans ---------------------------------------------------------------
 * diff[batch][n_species] diffusion coefficients d_s; params[batch][n_params]
 * reaction constants; w_ref[batch][n_species] the deviation origin or NULL
 * for the reaction's homogeneous equilibrium (zeros for TG_REACT_NONE).
 * tau > 0 is the time step.  Computes every phi_1 factor in FP64, rounds
 * it to the precision's storage type and uploads it; allocates two
 * state-sized scratch buffers.  Synchronous. */
int tg_plan_create(tg_grid g, int32_t n_species, int32_t batch, const double* diff,
                   int32_t reaction, int32_t n_params, const double* params,
                   const double* w_ref, double tau, int32_t precision, tg_plan* out);
int tg_plan_destroy(tg_plan p);
/* Number of state elements (batch * n_species * n1 * n2 * n3) and the
 * element size in bytes. */
int tg_plan_state_size(tg_plan p, int64_t* elems, int32_t* elem_bytes);
/* The reference state w_ref used by the plan, [batch][n_species]. */
int tg_plan_reference(tg_plan p, double* w_ref);

/* One step of the split exponential Euler method on `state` (in place).
 * Asynchronous: a non-finite value it writes is reported by the next
 * tg_run / tg_run_diag or by tg_sync_status. */
int tg_step(tg_plan p, void* state, void* stream);
/* Synchronise `stream` and report whether any update of this plan since the
 * last report wrote a non-finite value (TG_ENONFINITE; the flag is then
 * cleared).  For callers that step with tg_step / tg_step_diag. */
int tg_sync_status(tg_plan p, void* stream);
/* n_steps steps (in place): replays of captured HIP graphs of 32 and of 8
 * steps, then of 4, 2 and 1 step for the rest (all captured per state
 * pointer on the first run of 8 steps or more, or by tg_run_prepare, and
 * kept until the plan is destroyed or reconfigured); runs of fewer than 8
 * steps on a state without graphs launch directly; on route 4, resident
 * launches of up to 1024 steps.
 * Synchronises the stream at the end and returns TG_ENONFINITE if any
 * update produced a non-finite value. */
int tg_run(tg_plan p, void* state, int64_t n_steps, void* stream);
/* n_steps steps (in place) keeping the state before each one, for a reverse
 * sweep of the discrete adjoint (tg_adjoint_step) that recomputes nothing:
 * history (device, caller-owned, n_steps * the plan's state size elements,
 * the plan's layout) receives in slot k the state before step k, k = 0 ..
 * n_steps - 1, ahead of the step's launches: a device copy in the plan's
 * storage type, or, with history_fp64 != 0 and an FP32-storage plan, the
 * values widened to FP64 (for an FP64 reverse sweep of an FP32 forward).
 * history must not overlap state.  Steps launch directly (no graphs);
 * synchronises the stream at the end and returns TG_ENONFINITE as tg_run. */
int tg_run_history(tg_plan p, void* state, int64_t n_steps, void* history, int32_t history_fp64,
                   void* stream);
/* Capture (without running anything) the graphs tg_run replays for this
 * state pointer, so that a later tg_run spends no time capturing or
 * instantiating them.  Nothing to do on route 4.  Host-synchronous; the
 * graphs are dropped when the route or tiles change, as tg_run's are. */
int tg_run_prepare(tg_plan p, void* state);

/* Steady-state indicators (Section 5.2, the text after the disk experiment:
 * the integral mean of the solution and the L2 norm of one step's
 * increment), gathered in the step's last launch where the old and new
 * values meet, plus one small launch that adds up per-tile partial sums in
 * a fixed order (the results are reproducible run to run).
 *
 * Quadrature: each point owns the cell between the midpoints to its
 * neighbours along every coordinate (the end cells closed at 0 and rho_*,
 * 0 and pi, 0 and z_*; theta cells 2 pi / n wide), weighted by that cell's
 * measure in the volume element (rho, rho_*^2 sin(phi), rho^2 sin(phi),
 * rho), so the weights sum to |Omega|.
 *
 * tg_step_diag: one step as tg_step; diag is a device pointer to
 * [batch][n_species][2] doubles, written on `stream`:
 *   diag[.][.][0] = sum(w (w_ref + W_{n+1})) / sum(w)    (integral mean)
 *   diag[.][.][1] = sqrt(sum(w (W_{n+1} - W_n)^2))        (increment)
 * The first call allocates a partial-sum buffer of (npts / 8 + 64) * 2
 * doubles per slab, kept by the plan; calls on one plan from different
 * streams must not overlap.  TG_ENOTSUP for a grouped run (not offered). */
int tg_step_diag(tg_plan p, void* state, double* diag, void* stream);
/* tg_step_diag for callers that cannot allocate (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same step
 * and indicators, bit for bit, but the per-tile partial sums live in the
 * library's static device scratch (16 MiB per GPU, held until the process
 * ends) instead of a buffer the plan allocates, and the call allocates
 * nothing.  Limit: 2 (n1 n2 n3 / 8 + 64) batch n_species doubles of
 * partial sums must fit the 16 MiB (e.g. the 64 x 64 x 128 ball with two
 * species needs 2.1 MB); larger plans get TG_EINVAL.  All calls on one GPU
 * share the scratch: calls that overlap in time on one GPU (other streams,
 * other threads) race and must be ordered by the caller.  Call with the
 * plan's device current. */
int tg_step_diag_noalloc(tg_plan p, void* state, double* diag, void* stream);
/* n_steps steps; after steps every, 2 every, ... records the indicators of
 * that step into diag[r][batch][n_species][2] (device memory for
 * n_steps / every records; may be NULL when that is 0).  The steps between records replay captured
 * graphs.  Synchronises and checks for non-finite values like tg_run. */
int tg_run_diag(tg_plan p, void* state, int64_t n_steps, int32_t every, double* diag, void* stream);

/* Bulk-surface Schnakenberg system (Section 5.5, eqs. (bulkballsys),
 * (bulkballnl)): u, v in a ball (plan `bulk`: TG_BALL, two species,
 * d = (1, delta), kinetics TG_REACT_SCHNAKENBERG_SCALED with gamma =
 * alpha_1) and r, s on its surface (plan `surface`: TG_SPHERE of the same
 * radius on the ball's (theta, phi) grid, two species, d = (1, epsilon),
 * TG_REACT_SCHNAKENBERG_SCALED with gamma = zeta_1), same batch and
 * precision.  coupling = {zeta1, zeta2, zeta3, eta1, eta2} (host).
 *
 * The Robin conditions du/dn = zeta1 (zeta2 r - zeta3 u) and
 * delta dv/dn = zeta1 (eta1 s - eta2 v) enter the ball's boundary row
 * through its ghost point: F_u += kappa zeta1 (zeta2 r - zeta3 u) and
 * F_v += kappa zeta1 (eta1 s - eta2 v) on the layer rho = rho_*, with
 * kappa = (2 / h)(1 + h / rho_*), h = rho_* / n_rho; the surface gets
 * F_r -= zeta1 (zeta2 r - zeta3 u), F_s -= zeta1 (eta1 s - eta2 v).  The
 * exchange is evaluated at t_n with the kinetics; then each side takes its
 * own split step (route 0 plans run route 2 here: the exchange is added by
 * a separate stencil launch).  States: each plan's layout, in place.
 *
 * Bulk-surface DIB system on the cylinder (Section 5.6, eqs. (bulkcylsys),
 * (bulkcylnl)): u, v in a cylinder (plan `bulk`: TG_CYLINDER, two species,
 * d = (1, delta), TG_REACT_LINEAR with (alpha1, alpha2, beta1, beta2), its
 * reference -- the Dirichlet data of the top disk -- (alpha2, beta2)) and
 * r, s on its bottom disk (plan `surface`: TG_DISK with the cylinder's
 * (n_rho, n_theta) and radius, d = (1, epsilon), TG_REACT_DIB with
 * (zeta1, ..., zeta5, eta1, ..., eta5)), same batch and precision.
 * coupling = {alpha3, beta3, -, -, -} (the last three are not read but must
 * be finite).  The flux conditions du/dz = zeta1 alpha3 p(u, r, s),
 * dv/dz = zeta1 beta3 q(v, r, s) at z = 0 enter A_z's Neumann row through
 * its ghost point: on the layer z = 0, F_u -= (2 / h_z) zeta1 alpha3 p and
 * F_v -= delta (2 / h_z) zeta1 beta3 q, h_z = z_* / n_z; the disk's DIB
 * kinetics take the cylinder's z = 0 values u, v.  Evaluated at t_n, then
 * one split step per domain, as above.
 * TG_EINVAL when the plans do not match as described. */
int tg_coupled_step(tg_plan bulk, tg_plan surface, void* bulk_state, void* surface_state, const double* coupling,
                    void* stream);
/* n_steps coupled steps, replayed from a captured graph of 8 steps (kept by
 * the bulk plan per pair of states and coupling constants); synchronises and
 * returns TG_ENONFINITE if either state received a non-finite value. */
int tg_coupled_run(tg_plan bulk, tg_plan surface, void* bulk_state, void* surface_state, const double* coupling,
                   int64_t n_steps, void* stream);

/* Reverse step of the discrete adjoint of tg_step (not in the paper; the
 * exact derivative of the discrete map).  With mu_s = tau S_s^T lambda_s,
 * S_s = phi_1(tau d_s M_1) ... phi_1(tau d_s M_d):
 *   lambda_s <- lambda_s + d_s M^T mu_s + sum_r (dg_r / dw_s)(W_n) mu_r,
 *   grad[s]         += tau <lambda_s, (dS_s/dd_s) F_s> + <mu_s, M W_n,s>
 *   grad[nslab + s] += sum over points of mu_s (the derivative with respect
 *                      to a constant source in species s' reaction: the
 *                      Schnakenberg and 3-species constants a and b; for
 *                      TG_REACT_SCHNAKENBERG_SCALED, dL/da = gamma times it)
 * where nslab = batch * n_species, F_s = d_s M W_n,s + g_s(W_n) and the
 * old lambda_s is used on the right.  state_n: the state at step n (input,
 * device, plan layout); lambda: dL/dW_{n+1} in, dL/dW_n out (device, same
 * layout); grad: device doubles [2 * nslab], accumulated.  Runs the
 * per-mode kernels in the plan's storage type (FP32 for split-bf16 plans)
 * and allocates an 8-state workspace (plus three doubles per slab and
 * block of 256 points for the gradient's partial sums, added in a fixed
 * order, so repeated sweeps give identical gradients) on first use.  The reference state
 * (and the cylinder's Dirichlet value) is held fixed. */
int tg_adjoint_step(tg_plan p, const void* state_n, void* lambda, double* grad, void* stream);

/* Test hooks for the pieces of one step (same layouts as the state):
 *   what = TG_APPLY_F:         out = d_s M in + g(in)     (the F stage)
 *   what = TG_APPLY_DIFFUSION: out = d_s M in
 *   what = TG_APPLY_REACTION:  out = g(in)
 * in and out must not overlap. */
int tg_apply_operator(tg_plan p, const void* in, void* out, int32_t what, void* stream);
/* out = phi_1(tau d_s M_1) ... phi_1(tau d_s M_d) in, per species. */
int tg_apply_split_phi1(tg_plan p, const void* in, void* out, void* stream);
/* Kernel route of a plan.  0 (default): fused launches -- the stencil and
 * reaction inside the first product's tile load, each eigen-basis
 * sandwich (x V^-1, Hadamard phi_1, x V) in one launch, and the theta
 * sandwich, the rho product and the update in one launch per (rho, theta)
 * plane when it fits in LDS (where that single launch would both read the
 * state for F and update it in place, as the disk's plane launch does,
 * plans with two or more species compute F in a launch of its own first:
 * one species' workgroup must not overwrite values another species'
 * workgroup still reads for the reaction).  2: the same fused products
 * after a separate stencil + reaction launch.  1: one launch per mu-mode
 * product plus the stencil launch.  3 (ball and cylinder, FP64 / FP32): as 1, but the mode
 * whose term is scaled by rho^-2 alone (the ball's phi, the cylinder's
 * theta) is applied by per-slice dense factors phi_1(tau d rho_i^-2 A), one
 * per radial index i (Section 4: phi_1 of the block-diagonal term, blockwise),
 * built on first selection; TG_ENOTSUP elsewhere.  4 (disk plans in FP64
 * or FP32 whose step is route 0's single plane launch): resident steps --
 * one workgroup per instance keeps the state, F and the sandwich
 * intermediate of every species in LDS and runs many steps per launch
 * (tg_run: up to 1024; tg_step: one), the reaction reading the other
 * species from the same LDS; TG_ENOTSUP where the species' tiles of an
 * instance do not fit in LDS together (160 KB) or the step has another
 * shape.  Steps with indicators (tg_step_diag) run route 0's launches.
 * Routes 0 and 2 fall back to 1 where a shape does not fit in LDS; a
 * column width set by tg_plan_set_tiles that the new route's in-tile
 * stencil does not fit goes back to 16.  All routes compute the same
 * step.  tg_plan_autotune also tries routes 3 and
 * 4 where they exist. */
int tg_plan_set_route(tg_plan p, int32_t route);
/* The route actually used by tg_step / tg_run (after fall-back). */
int tg_plan_route(tg_plan p, int32_t* route);
/* Number of launches of the active route's split chain (in application
 * order, eqs. (ee_*)); if modes != NULL the mode mu of the leading product
 * of each launch, and if flops != NULL its algorithmic flop count (2 n_mu
 * per output element of every mu-mode product it performs). */
int tg_plan_chain(tg_plan p, int32_t* n_ops, int32_t* modes, double* flops);
/* Benchmark / test hook: run launch `op` (0-based) of the active route's
 * split chain alone.  Route 1: out = in x_mu L (with its Hadamard phi_1
 * factor where the chain has one).  Routes 0 and 2: as in a step, `in`
 * being the previous launch's output, except for the first launch of route
 * 0, which reads the state and evaluates F = d M W + g(W) itself.  Route 4:
 * route 0's single fused launch.  A final update is replaced by a store. */
int tg_apply_chain_op(tg_plan p, int32_t op, const void* in, void* out, void* stream);

/* Benchmark hook: n_steps steps of tg_step (direct launches, no graph) with
 * a HIP event recorded on the stream before every kernel launch and after
 * each step's last one.  launch_us[l] (l < *n_launches <= max_launches) is
 * the average time from the end of launch l-1 (or of the previous step) to
 * the end of launch l: the kernel's duration plus its dispatch gap.
 * Creates 1 + launches-per-step events per step for the duration of the
 * call; synchronous. */
int tg_run_timed(tg_plan p, void* state, int64_t n_steps, void* stream, int32_t max_launches,
                 int32_t* n_launches, double* launch_us);

/* ---- batching ----------------------------------------------------------
 * Grouped run (not in the paper; it batches many instances of the problem
 * of Section 2, e.g. parameter sweeps on grids of different sizes).
 * plans[0 .. n_plans), 1 <= n_plans <= 4, each with its own distinct state
 * (device, plan layout, updated in place): n_steps steps of every plan.
 * When all plans share the precision (FP64 or FP32), the route (0 or 2)
 * and the kinds of their fused launches, launch k of a step covers the
 * tiles of every plan in ONE persistent launch (grid = occupancy x CUs,
 * tiles remapped so each XCD walks a contiguous range); otherwise the
 * plans' launches follow each other.  Steps are replayed from a graph
 * captured on first use per (plans, configurations, states) and kept by
 * plans[0] until it is destroyed; when a plan is on route 4, every plan
 * runs its n_steps as tg_run would (resident launches, or its own graph
 * replays), one plan after the other.  Synchronises the stream at the end;
 * TG_ENONFINITE if any plan produced a non-finite value. */
int tg_group_run(const tg_plan* plans, int32_t n_plans, void* const* states, int64_t n_steps,
                 void* stream);
/* For the same arguments: whether the launches are grouped (1) or per
 * plan (0), and the kernel launches per step.  Builds the group if needed. */
int tg_group_info(const tg_plan* plans, int32_t n_plans, void* const* states, int32_t* grouped,
                  int32_t* launches_per_step);

/* Route for a grouped run: times `iters` grouped steps (after 2 warm-up
 * steps) with every plan on route 0, on route 2, and on route 2 with the
 * 16-column strided launches without a plane tail widened to 32 columns
 * where that fits (only route 0's in-tile stencil held them at 16), on
 * private copies of the states (not modified), and sets the fastest
 * (by at least 2%) on all plans, so that they stay groupable.  Plans whose fused route does
 * not fit are left as they are (*best_us = 0).  Allocates one copy of each
 * state for the duration of the call; synchronous. */
int tg_group_autotune(const tg_plan* plans, int32_t n_plans, void* const* states, int32_t iters, void* stream,
                      double* best_us);

/* ---- autotuning ----------------------------------------------------------
 * Times `iters` steps (after 2 warm-up steps) of each candidate launch
 * configuration on a private copy of `state` (device, plan layout; not
 * modified) and keeps the fastest: the route (0, 2, and 1 except for
 * split-bf16 plans; 3 and 4 where they exist) and, per fused launch, the
 * tile width (16 / 32 / 64 columns for strided launches that do not cover
 * whole planes, 16 / 32 rows for first-mode launches), by coordinate
 * descent; a candidate must be at least 2% faster to replace the current
 * choice (routes are tried in the order 0, 2, 1, 3, 4).  Routes 0 to 3 are
 * timed by direct launches of single steps, route 4 by one resident launch
 * of `iters` steps, as tg_run runs them (its single steps, tg_step, cost a
 * launch each and more than route 0's).  Every candidate computes the same
 * step.
 * *best_us: time per step of the choice.
 * Allocates one state-sized buffer for the duration of the call;
 * synchronous.  Captured graphs of the plan are dropped. */
int tg_plan_autotune(tg_plan p, const void* state, int32_t iters, void* stream, double* best_us);
/* Tile width of each fused launch (columns for strided launches, rows for
 * first-mode launches); *n_ops = number of fused launches. */
int tg_plan_tiles(tg_plan p, int32_t* n_ops, int32_t* tiles);
/* Set the tile widths (n_ops = number of fused launches; 16 / 32 rows for
 * first-mode launches, 16 or a multiple of 32 columns for strided ones;
 * launches that cover whole planes keep theirs).  TG_EINVAL, nothing
 * changed, if a width is not allowed or does not fit in LDS as the active
 * route launches it: route 0 computes F inside the first launch's tile
 * load, which also needs LDS for the stencil's neighbours, route 2 does
 * not, so route 2 can take wider first tiles.  tg_plan_set_route to a
 * route whose in-tile stencil does not fit a width set before puts that
 * launch back to 16 columns. */
int tg_plan_set_tiles(tg_plan p, int32_t n_ops, const int32_t* tiles);

#ifdef __cplusplus
}
#endif

#endif /* TGEXP_H */
