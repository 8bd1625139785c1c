/*
 * lb2d.h -- C ABI of the MI355X (gfx950) library for 2-D lattice Boltzmann
 * simulations with the commands of "Introduction to Perl module lb2d.pm 0.1
 * for basic Lattice Boltzmann simulations" (D. Sergi, arXiv:1202.0442).
 *
 * Conventions (every entry point):
 *  - Returns an int status: LB2D_OK (0) or one of the negative LB2D_E_*
 *    codes below; lb2d_last_error() gives a message.  Nothing aborts: where
 *    the paper stops a simulation with an error message on a wrong command
 *    order, the call returns LB2D_E_ORDER and leaves the context
 *    unchanged.
 *  - Sizes are NODE COUNTS nx, ny (x fastest).  The paper's
 *    lattice(d2q9, Nx, Ny, tau) numbers its sites 0..Nx, 0..Ny, i.e. it has
 *    Nx+1 by Ny+1 nodes; callers that follow the paper pass Nx+1, Ny+1.
 *  - Host arrays are row-major [ny][nx] (x fastest), owned by the caller,
 *    read or written only during the call.
 *  - Device memory is owned by the caller: lb2d_workspace_bytes() says how
 *    much one lattice needs, lb2d_bind() hands over a device pointer and a
 *    HIP stream.  The caller keeps that memory alive until lb2d_destroy()
 *    (or a new bind).  The library allocates no device memory.
 *  - All device work is enqueued on the bound stream.  lb2d_iteration()
 *    returns without waiting; read-outs and budgets synchronise the stream.
 *  - Velocity numbering (D2Q9): e0=(0,0), e1=(1,0), e2=(0,1), e3=(-1,0),
 *    e4=(0,-1), e5=(1,1), e6=(-1,1), e7=(-1,-1), e8=(1,-1).  A "mode" in
 *    aveforce/aveacceleration is one of 0..8 (the paper's "e0".."e8").
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef LB2D_H
#define LB2D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LB2D_OK 0
#define LB2D_E_INVAL (-1)       /* bad argument value */
#define LB2D_E_ORDER (-2)       /* command order rule of the paper violated */
#define LB2D_E_UNSUPPORTED (-3) /* a form of a command this library lacks */
#define LB2D_E_STATE (-4)       /* not bound yet / already bound / running */
#define LB2D_E_HIP (-5)         /* a HIP runtime call failed */
#define LB2D_E_SIZE (-6)        /* workspace too small or size overflow */

/* Storage formats of the populations (arithmetic is FP64 for LB2D_F64 and
 * FP32 otherwise).  Populations are stored as deviations f_i - w_i rho_ref
 * (rho_ref = mean initial density); the 16-bit formats also scale each
 * direction by a power of two (2, 8, 32 for rest, axis, diagonal) and round
 * to nearest even.  Deposits and budgets are always FP64. */
#define LB2D_F64 0
#define LB2D_F32 1
#define LB2D_F16 2
#define LB2D_BF16 3

/* Budget vector of lb2d_budgets(), FP64. */
#define LB2D_NBUDGET 16
#define LB2D_B_MASS0 0          /* sum of rho_1 over fluid nodes */
#define LB2D_B_MASS1 1          /* sum of rho_2 over fluid nodes */
#define LB2D_B_MOMX 2           /* sum over comps and fluid nodes of j_x */
#define LB2D_B_MOMY 3           /*   (post-collision momentum)          */
#define LB2D_B_SOLUTE 4         /* sum of C over fluid nodes */
#define LB2D_B_DEPOSIT 5        /* sum of b over solid nodes */
#define LB2D_B_REMOVED0 6       /* fluid-1 mass of nodes that turned solid */
#define LB2D_B_REMOVED1 7       /* fluid-2 mass of nodes that turned solid */
#define LB2D_B_REMOVED_C 8      /* solute of nodes that turned solid */
#define LB2D_B_INFLOW 9         /* solute injected by the x openings */
#define LB2D_B_OUTFLOW 10       /* solute that left through the x openings */
#define LB2D_B_STEPS 11         /* completed time steps */
#define LB2D_B_GROWN 12         /* nodes that turned solid by growth */
#define LB2D_B_FLUID 13         /* current number of fluid nodes */
#define LB2D_B_CONSUMED 14      /* deposits reset to zero by growth */

typedef struct lb2d_ctx lb2d_ctx;
typedef struct lb2d_batch lb2d_batch;

/* ------------------------------------------------------------ lifetime */

/* New empty context on HIP device `hip_device`.  *out receives it. */
int lb2d_create(lb2d_ctx **out, int hip_device);
/* Waits for the work queued on the bound stream, then frees the context
 * and its graphs (not the caller's device memory, which may be freed once
 * this returns). */
int lb2d_destroy(lb2d_ctx *ctx);
/* Message of the last failed call on ctx ("" if none; static text for a
 * NULL ctx). */
const char *lb2d_last_error(const lb2d_ctx *ctx);

/* ---------------------------------------------- initialization commands */

/* lattice command (Sec. "Commands", lattice): style must be "d2q9"; nx, ny
 * node counts >= 3; tau > 1/2 the relaxation time.  Must come first; the
 * box is periodic on both axes unless openings say otherwise. */
int lb2d_lattice(lb2d_ctx *ctx, const char *style, int nx, int ny, double tau);

/* fluids command: two components with relaxation times tau1, tau2 > 1/2
 * and density-ratio parameters alpha1, alpha2 in [0,1) (pass NaN for the
 * default 4/9, which gives the plain equilibrium Eq. (eq)).  The
 * equilibrium is w_i rho [A_i + 3 e.u + 9/2 (e.u)^2 - 3/2 u.u] with
 * A_0 = (9/4) alpha, A_i = (9/5)(1 - alpha).  After lattice, before any
 * force and before bind. */
int lb2d_fluids(lb2d_ctx *ctx, double tau1, double tau2, double alpha1,
                double alpha2);

/* solute command: one solute species with relaxation time tau_s > 1/2,
 * advected by the solvent velocity of Eq. (u_solvent), on
 *   q = 9: D2Q9, g_eq = w_i C (1 + 3 e.u), D = (tau_s - 1/2)/3, or
 *   q = 4: the paper's D2Q4 (directions e1..e4), g_eq = C/4 (1 + 2 e.u),
 *          D = (tau_s - 1/2)/2.
 * Other q: LB2D_E_INVAL.  Needs the general (FP64/FP32) step. */
int lb2d_solute(lb2d_ctx *ctx, double tau_s, int q);

/* inlet/outlet + inlet_solute/outlet_solute commands: nodes lo..hi
 * (inclusive, along the wall) of wall "xlo", "xhi", "ylo" or "yhi" are a
 * solute opening; kind "inlet" or "outlet".  Styles:
 *   "dirichlet": C = value after streaming; the unknown populations share
 *                the deficit value - C' in proportion to their weights (a
 *                single unknown takes all of it, as printed);
 *   "adiabatic": zero normal flux, each unknown copies its mirror across
 *                the wall (g3 = g1 on xhi);
 *   "flux":      C = (v C0 + D C1)/(D + v) at an inlet and
 *                (v C0 - D C1)/(v - D) at an outlet (App. B), C0 = value,
 *                v > 0 the velocity of the injected solution (v != D at an
 *                outlet, where the rule is singular), D the solute
 *                diffusivity, C1 the concentration of the next node inward
 *                at the previous time level; all populations of the node
 *                are set to their equilibrium at C.
 * An opening on a wall makes the solute non-periodic along that axis; the
 * parts of the axis' two walls outside openings are impermeable to the
 * solute (bounce-back).  The fluid stays periodic.  At most 8 openings,
 * no node on two.  Needs solute; before bind. */
int lb2d_solute_opening_range(lb2d_ctx *ctx, const char *wall, int lo, int hi,
                              const char *kind, const char *style, double value,
                              double v);
/* The whole x wall "xlo" (inlet) or "xhi" (outlet) as a "dirichlet" or
 * "adiabatic" solute opening (lb2d_solute_opening_range with lo = 0,
 * hi = ny - 1). */
int lb2d_solute_opening(lb2d_ctx *ctx, const char *wall, const char *style,
                        double value);

/* inlet/outlet + inlet_momentum/outlet_momentum commands: nodes lo..hi
 * (inclusive, along the wall) of wall "xlo", "xhi", "ylo" or "yhi" are an
 * opening for fluid component comp; kind "inlet" or "outlet".  Styles:
 *   "poiseuille": velocity along the wall normal with the paper's profile
 *       v(k) = 4 v / L^2 [(L/2)^2 - ((2k - lo - hi)/2)^2], L = hi - lo + 1
 *       (v = v_max);
 *   "uniform":    velocity v along the wall normal;
 *   "dirichlet":  density (pressure rho/3) rho held;
 *   "gradient":   after the collision f(wall) = 2 f(wall+n) - f(wall+2n).
 * Velocities point into the domain for inlets and out of it for outlets;
 * the tangential velocity is zero.  The Zou-He closure (App. A) sets the
 * three populations entering the domain after streaming and bounce-back;
 * the opening nodes then collide as usual.  rho is also the density the
 * opening nodes start with (velocity styles also start at their velocity).
 * Openings override the periodic wrap only on their own nodes.  Up to 8
 * openings; a node may belong to one opening per component; |v| < 1,
 * rho > 0.  After lattice (and fluids), before bind. */
int lb2d_momentum_opening(lb2d_ctx *ctx, const char *wall, int lo, int hi, int comp,
                          const char *kind, const char *style, double v,
                          double rho);

/* boundary_style command (Commands section, boundary_style; Fig. slip).
 * Must precede every obstacle; sets how the solids of the obstacles that
 * follow, and the solids made by growth, treat a fluid population that
 * hits them:
 *   "noslip": half-way bounce-back (R = 0);
 *   "slip":   a diagonal mode that hits a flat wall is mirrored and goes on
 *             forward (R = 1); at a corner, or when the node it would land
 *             on is solid, it bounces back; axis modes always bounce back;
 *   "mixed":  a share R (0 <= R <= 1, the argument) goes forward by the
 *             slip rule and 1 - R bounces back;
 *   "hybrid": each obstacle carries its own style (lb2d_obstacle_style);
 *             solids made by growth are noslip.
 * R is read only by "mixed".  The solute always bounces back (or reacts).
 * The step reads every solid's R per component: one FP64 array per
 * component on the device.  Returns LB2D_E_INVAL for an unknown style or
 * an R outside [0, 1]. */
int lb2d_boundary_style(lb2d_ctx *ctx, const char *style, double R);

/* Per-obstacle style of the hybrid boundary style (obstacle command's
 * extra arguments, one style per component): component comp of the
 * obstacles that follow uses "noslip", "slip" or "mixed" with share R.
 * Only after boundary_style("hybrid") (LB2D_E_ORDER otherwise); comp must
 * name a component of the fluids command. */
int lb2d_obstacle_style(lb2d_ctx *ctx, int comp, const char *style, double R);

/* Rounding of 16-bit population storage (an extension; the paper stores
 * FP64): "nearest" (round to nearest even, the default) or "stochastic"
 * (round up or down with probabilities given by the distance to the two
 * neighbouring 16-bit values, using the gfx950 hardware converts and a
 * counter-based hash of (seed, step, node, and in the general step the
 * plane group: component 0, component 1, solute)).  Stochastic rounding
 * keeps per-step changes smaller than half an ulp on average, so slowly
 * forced flows do not stall and near-steady states do not drift in mass;
 * runs stay bitwise reproducible for a given seed.  The step kernels round
 * this way; populations written outside them (initial fields, gradient
 * openings, lb2d_set_populations) round to nearest.
 * Before bind; at bind, "stochastic" needs FP16 or BF16 storage
 * (LB2D_E_UNSUPPORTED otherwise) and population arrays below 4 GiB
 * (LB2D_E_SIZE).  A batch of such lattices rounds as each would alone. */
int lb2d_rounding(lb2d_ctx *ctx, const char *mode, uint64_t seed);

/* obstacle command, rectangle: nodes x0..x1, y0..y1 (inclusive,
 * 0 <= x0 <= x1 < nx, 0 <= y0 <= y1 < ny) become solid. */
int lb2d_obstacle_rect(lb2d_ctx *ctx, int x0, int x1, int y0, int y1);
/* obstacle command, circle: node (x,y) is solid when dx^2 + dy^2 <= r^2,
 * dx, dy integer minimum-image distances on the periodic box (compared in
 * FP64).  0 <= xc < nx, 0 <= yc < ny, r >= 0. */
int lb2d_obstacle_circle(lb2d_ctx *ctx, int xc, int yc, double r);
/* obstacle from a host byte map (nonzero = solid), OR-ed into the mask. */
int lb2d_obstacle_mask(lb2d_ctx *ctx, const uint8_t *host_mask);

/* surface_reaction command: D dC/dn = kr (C - Cs) on solid surfaces, style
 * "growth"; every solid starts with deposit b0; a solid whose deposit
 * exceeds bmax turns one of its direct fluid neighbours (E,N,W,S, not on an
 * open solute column) solid, chosen by a counter-based SplitMix64 hash of
 * (seed, step, node), and its deposit resets to 0.  Per link i the rate is
 * k_i = kr w_i / W (W = 1/6 on D2Q9, 1/4 on D2Q4); the link concentration
 * C_i = (2 g_out + k_i Cs) / (2 w_i + k_i) and returning population
 * 2 w_i C_i - g_out are, on D2Q4, the paper's rule of App. C.  Deposits
 * are FP64.  Needs solute; kr >= 0. */
int lb2d_surface_reaction(lb2d_ctx *ctx, double kr, double Cs,
                          const char *style, double b0, double bmax,
                          uint64_t seed);

/* position0 / momentum0: initial density and velocity of component comp
 * (0 or 1), host arrays of nx*ny doubles (ux, uy may be NULL = 0).  The
 * populations start at their equilibrium (Fig. "algorithm").  Components
 * never set start at rho = 1, u = 0.  Densities must be positive and
 * finite, velocities finite (LB2D_E_INVAL).  Before bind. */
int lb2d_set_fields(lb2d_ctx *ctx, int comp, const double *rho,
                    const double *ux, const double *uy);
/* concentration0: initial solute concentration (nx*ny doubles) and the
 * velocity of its equilibrium (NULL = 0), all finite (LB2D_E_INVAL).
 * Default C = 0.  Needs solute. */
int lb2d_set_concentration(lb2d_ctx *ctx, const double *C, const double *ux,
                           const double *uy);

/* -------------------------------------------------- force field commands */

/* aveforce command: adds value * e_mode to the force on component comp
 * (0 or 1) at every fluid node; repeated calls sum.  After lattice/fluids,
 * before bind. */
int lb2d_aveforce(lb2d_ctx *ctx, int mode, double value, int comp);
/* aveacceleration command: adds value * e_mode to the acceleration of comp;
 * the force is rho_comp times the summed acceleration. */
int lb2d_aveacceleration(lb2d_ctx *ctx, int mode, double value, int comp);
/* interforce command (Shan-Chen cohesion, computed from the densities
 * after streaming of the same step).  Two-component form (psi0 and rho0
 * NaN): F_c = -G rho_c(x) sum_{i=1..8} w_i rho_cbar(x + e_i) e_i, cbar the
 * other component.  One-component form (one fluid; psi0 > 0 and rho0 > 0
 * given): F = -G psi(x) sum_{i=1..8} w_i psi(x + e_i) e_i with
 * psi = psi0 exp(-rho0 / rho).  Densities and psi are 0 on solids.
 * LB2D_E_INVAL for a form that does not match the number of fluids. */
int lb2d_interforce(lb2d_ctx *ctx, double G, double psi0, double rho0);
/* adhesiveforce command.  Two-component form (psi0, rho0 NaN):
 * F_c += -G_c rho_c(x) sum_{i=1..8} w_i s(x + e_i) e_i (s = 1 on solids).
 * One-component form (one fluid, comp 0, psi0 and rho0 of its own):
 * F += -G psi(x) sum_{i=1..8} w_i s(x + e_i) e_i. */
int lb2d_adhesiveforce(lb2d_ctx *ctx, double G, double psi0, double rho0,
                       int comp);

/* intersolute command: adds tau_s F / C to the solvent velocity in the
 * solute equilibrium, with F = -G psi(x) sum_{i=1..4} psi(x + e_i) e_i
 * over the four axis neighbours (no lattice weights) and
 * psi = psi0 exp(-C0 / C).  The concentrations are those of the same step
 * after streaming (as for interforce); psi is 0 on solids, where C <= 0
 * and across a wall of a non-periodic solute axis, and the term is added
 * only where C > 0.  Needs the solute command (LB2D_E_ORDER otherwise);
 * G and psi0 finite, C0 > 0 (LB2D_E_INVAL).  Before bind. */
int lb2d_intersolute(lb2d_ctx *ctx, double G, double psi0, double C0);

/* ------------------------------------------------------------- memory */

/* Bytes of device memory one lattice needs with the given storage format
 * (LB2D_F64/F32/F16/BF16), after all commands above.  Every lattice can
 * store FP16 or BF16 (FP32 arithmetic), rounded to nearest or
 * stochastically; stochastic rounding of FP32 or FP64 storage is
 * LB2D_E_UNSUPPORTED. */
int lb2d_workspace_bytes(lb2d_ctx *ctx, int storage, size_t *bytes);
/* Binds `bytes` of caller device memory at dev_ptr (256-byte aligned,
 * on the context's device) and the HIP stream `hip_stream` (NULL = the
 * null stream) with the storage chosen in the last lb2d_workspace_bytes
 * call; rasterises obstacles and sets the initial populations on the GPU.
 * After this, commands return LB2D_E_STATE. */
int lb2d_bind(lb2d_ctx *ctx, void *dev_ptr, size_t bytes, void *hip_stream);

/* ------------------------------------------------------------ action */

/* iteration command: advances nsteps >= 0 time steps (stream with
 * bounce-back, moments, forces, collision; then solute stream, reactive and
 * opening rules, collision, deposit, growth).  Asynchronous on the stream;
 * launches captured HIP graphs: graphs of 60 steps, then one graph of the
 * remaining steps (a single launch for one step).  A graph is captured the
 * first time its length and starting parity (even or odd step count) are
 * needed, uploaded to the device on the context's stream and kept.  Inside the graphs, a one-fluid lattice (no solute, no
 * Shan-Chen, no openings or slip solids) of at least 72 x 24 nodes (40 x 24
 * in FP64) advances by a multi-step kernel, five steps per launch (the first
 * four of each five are kept in LDS and never reach memory), then single
 * steps for the remainder; the results equal single steps bit for bit. */
int lb2d_iteration(lb2d_ctx *ctx, int64_t nsteps);
/* Steps that one launch of the dominant step kernel advances inside the
 * graphs of lb2d_iteration: 5 for the multi-step kernel, else 1. */
int lb2d_steps_per_launch(lb2d_ctx *ctx, int *steps);
/* Captures and uploads, without running any step, the graphs that
 * lb2d_iteration(ctx, nsteps) will launch from the current step count, so
 * that the call itself launches without capture or upload cost (for timed
 * regions). */
int lb2d_prepare(lb2d_ctx *ctx, int64_t nsteps);

/* ------------------------------------------------------------ output */

/* output command, fluid part: density and velocity of component comp (or
 * of the mixture, comp = -1) after the last collision, velocity including
 * half the force, (j_post - F/2) / rho.  Solid nodes read rho = -11 and
 * u = 0.  Host arrays of nx*ny doubles. */
int lb2d_moments(lb2d_ctx *ctx, int comp, double *rho, double *ux,
                 double *uy);
/* output command, solute part: C on fluid nodes (0 on solids) and deposit
 * b on solid nodes (0 on fluid nodes); either pointer may be NULL. */
int lb2d_solute_state(lb2d_ctx *ctx, double *C, double *b);
/* Current solid mask (1 = solid), nx*ny bytes. */
int lb2d_mask(lb2d_ctx *ctx, uint8_t *m);
/* thermo command: FP64 budgets, out[LB2D_NBUDGET] (see LB2D_B_*). */
int lb2d_budgets(lb2d_ctx *ctx, double *out);
/* lb2d_budgets for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid allocation): the
 * same kernels and results, bit for bit, but the reduction's scratch (per-row
 * partials, sums, tally totals) lives in a 4 MiB device array of the library
 * instead of the bound workspace; the call allocates nothing.  Lattices of
 * more than 65533 rows return LB2D_E_SIZE.  Every call on one GPU shares that
 * GPU's array (each value read is written in the same call, so nothing
 * carries over), so calls that overlap on one GPU, from several threads or
 * streams, race. */
int lb2d_budgets_noalloc(lb2d_ctx *ctx, double *out);

/* Raw state, decoded to FP64 f_i (comp 0/1) or g_i (comp -1): 9*nx*ny
 * doubles [9][ny][nx] of the post-collision state (for checkpoints and
 * one-step comparisons).  set encodes into the storage format.  With a
 * D2Q4 solute, planes 0 and 5..8 of g read as 0 and must be 0 on set
 * (LB2D_E_INVAL otherwise). */
int lb2d_get_populations(lb2d_ctx *ctx, int comp, double *out);
int lb2d_set_populations(lb2d_ctx *ctx, int comp, const double *in);
/* Raw deposit array (nx*ny doubles, all nodes) and step counter. */
int lb2d_get_deposit(lb2d_ctx *ctx, double *b);
int lb2d_set_deposit(lb2d_ctx *ctx, const double *b);
/* Replaces the solid mask (nx*ny bytes, 1 = solid; for checkpoints) and
 * rebuilds the link words; pending growth triggers are cleared.  The
 * reflected shares of slip/mixed solids are not changed: a node made solid
 * here keeps the share it last had (0, noslip, if it never was solid). */
int lb2d_set_mask(lb2d_ctx *ctx, const uint8_t *m);
/* Steps completed since bind. */
int lb2d_step_count(lb2d_ctx *ctx, int64_t *t);

/* Checkpoint and restart (the binary counterpart of the paper's
 * write_restart / read_data commands).  lb2d_checkpoint_bytes gives the
 * size; lb2d_checkpoint_save copies the lattice's whole device state
 * (populations, mask, link words, deposits, growth triggers, running
 * tallies, step counters) and its step count into the caller's host buffer
 * (waits for the bound stream); lb2d_checkpoint_load restores such a buffer
 * into a lattice bound after the same commands with the same storage and
 * rounding (LB2D_E_INVAL if the saved lattice's sizes, components, solute,
 * storage, rounding, population shift or workspace layout differ; the
 * other parameters are the caller's to match; LB2D_E_SIZE if the data is
 * truncated).  Continuing after a load gives the run that was saved, bit
 * for bit. */
int lb2d_checkpoint_bytes(lb2d_ctx *ctx, size_t *bytes);
int lb2d_checkpoint_save(lb2d_ctx *ctx, void *host, size_t bytes);
int lb2d_checkpoint_load(lb2d_ctx *ctx, const void *host, size_t bytes);

/* ------------------------------------------------------- batched lattices */

/* A batch advances many bound one-fluid lattices (no solute, no Shan-Chen;
 * each with its own size, geometry, tau and forces, one storage format) in
 * one launch per time step, or per five steps: blocks walk a table of
 * tiles of all the lattices.  The tile shape (one, two or four brick rows of
 * the one-step kernel's 256-thread blocks: 64x4, 32x8 or 16x16 nodes for
 * FP32/FP64, 32x8, 16x16 or 8x32 for 16-bit storage; or the multi-step
 * kernel's 64x16 tile, 32x16 for FP64, when every lattice has at least that
 * extent plus four nodes each way), the
 * order of the tiles in the table and the grid (one block per tile or
 * persistent blocks) are picked by an autotuner at finalize; results never
 * depend on them. */
int lb2d_batch_create(lb2d_batch **out, int hip_device);
/* Waits for the batch's queued work, then frees the batch (not its
 * lattices, nor the caller's device memory). */
int lb2d_batch_destroy(lb2d_batch *b);
const char *lb2d_batch_last_error(const lb2d_batch *b);
/* Adds a bound lattice (the batch does not own it).  All lattices of a
 * batch share one storage format and one rounding mode (LB2D_E_INVAL
 * otherwise); with stochastic rounding each keeps its own seed and step
 * count, so a batched run equals the lattices stepped one by one, bit for
 * bit. */
int lb2d_batch_add(lb2d_batch *b, lb2d_ctx *lattice);
/* Device bytes for the batch's tables (after all adds). */
int lb2d_batch_workspace_bytes(lb2d_batch *b, size_t *bytes);
/* Binds the tables' memory and the stream, builds the tile tables, runs the
 * autotuner (timed trial steps that write only the lattices' next-step
 * buffers, leaving their state unchanged) unless tune_cache_json names a
 * readable file holding a previous choice for the same lattice set, in which
 * case that choice is used; the choice is written back to that file when
 * the path is not NULL.  Stream NULL = null stream. */
int lb2d_batch_finalize(lb2d_batch *b, void *dev_ptr, size_t bytes,
                        void *hip_stream, const char *tune_cache_json);
/* Advances every lattice by nsteps (asynchronous, graph-launched). */
int lb2d_batch_iteration(lb2d_batch *b, int64_t nsteps);
/* The tuned launch shape: tile width, tile height, schedule id (0 lattice
 * by lattice, 1 largest lattices first, 2 tiles of all lattices interleaved
 * round-robin), blocks per CU (0 = one block per tile). */
int lb2d_batch_config(lb2d_batch *b, int *tile_w, int *tile_h, int *schedule,
                      int *blocks_per_cu);
/* Steps one launch of the batch's step kernel advances: 5 when the
 * autotuner chose the multi-step kernel's tile, else 1. */
int lb2d_batch_steps_per_launch(lb2d_batch *b, int *steps);
/* The autotuner's trials at finalize: *count receives their number (0 when
 * the choice came from the tune cache); the first min(max, count) are
 * written to the caller's arrays of max entries: tile width and height,
 * schedule id, blocks per CU and the measured milliseconds per step.
 * max = 0 only queries the count. */
int lb2d_batch_trials(lb2d_batch *b, int max, int *tile_w, int *tile_h,
                      int *schedule, int *blocks_per_cu, double *ms,
                      int *count);

/* -------------------------------------------------------- measurement */

/* Average device time per call, in milliseconds, of the dominant kernel of
 * the last lb2d_iteration / lb2d_batch_iteration measured with HIP events
 * on the bound stream when timing is on (lb2d_set_timing(ctx, 1)); timing
 * launches the steps one by one instead of through graphs. */
int lb2d_set_timing(lb2d_ctx *ctx, int on);
int lb2d_kernel_time(lb2d_ctx *ctx, double *ms_per_launch, int64_t *launches);

/* Plain device-to-device copy of `bytes` (a multiple of 16; src and dst
 * device memory, not overlapping) repeated `reps` times on the stream;
 * *ms = average milliseconds per copy.  Not a command of the paper: it
 * measures the practical HBM ceiling the stencil is compared with. */
int lb2d_copy_bench(void *src, void *dst, size_t bytes, int reps, void *hip_stream, double *ms);

#ifdef __cplusplus
}
#endif
#endif /* LB2D_H */
