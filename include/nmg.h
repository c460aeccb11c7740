/*
 * nmg.h -- C ABI of the MI355X (gfx950) Newton multigrid library for steady
 * shallow water equations with topography and wet/dry areas, after
 * K. Wu and H. Tang, "A Newton multigrid method for steady-state shallow
 * water equations with topography and dry areas" (arXiv:1608.06721).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Arrays.  Every array argument is a DEVICE pointer to caller-owned FP64
 * memory (for example a torch.cuda tensor) unless its name ends in _host.
 * Cell vectors use the layout v[c][ny][nx] (x fastest, component-major),
 * c < NC with NC = 2 in 1D (h, hu) and NC = 3 in 2D (h, hu, hv); the bed is
 * z[ny][nx].  Block matrices use A[b][r][c][ny][nx]: block b in the order
 * D, W, E, S, N (1D: D, W, E) couples cell (i, j) to itself or to its west,
 * east, south or north neighbour; A[b][r][c] at cell (i, j) is the
 * derivative of row r of cell (i, j)'s equation with respect to component c
 * of that neighbour's unknown.  Blocks that point out of the grid are zero.
 *
 * Ownership.  The library never frees caller memory.  It owns only the
 * workspace inside the opaque context (the multigrid hierarchy in a
 * colour-split layout, about 1.33 x 2 x (45 + 6) x 8 bytes per 2D cell).
 *
 * Streams.  All work is enqueued on the HIP stream given to nmg_create and
 * is stream-ordered with the caller's work on that stream.  Entry points
 * that return values to host memory (res_l1_host, stats) synchronize that
 * stream.  A context must not be used from two threads at once.
 *
 * Errors.  Every function returns NMG_OK (0) or a status below; no
 * exception crosses the ABI.  nmg_last_error gives a message for the last
 * failure on a context.  On NMG_EHIP the context should be destroyed.
 *
 * Floating point.  All arithmetic is IEEE FP64 without contraction; each
 * expression is evaluated in a fixed documented order, so results are
 * deterministic run to run and for any launch shape.
 */
#ifndef NMG_H
#define NMG_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nmg_ctx nmg_ctx;

enum {
    NMG_OK = 0,
    NMG_NOT_CONVERGED = 1,   /* max_newton reached; U holds the last iterate */
    NMG_EINVAL = -1,         /* bad argument (grid, BC, params, level, null pointer) */
    NMG_ENOMEM = -2,         /* device allocation failed */
    NMG_EHIP = -3,           /* a HIP runtime call failed */
    NMG_ENONFINITE = -4,     /* a residual became NaN/Inf; U holds the last finite iterate */
    NMG_EDIVERGED = -5       /* sum ||R_i||_1 grew beyond 1e8 x its first value */
};

enum { NMG_FLUX_HLL = 0, NMG_FLUX_LLF = 1, NMG_FLUX_HLLC = 2 /* 2D only */ };
enum { NMG_BC_REFLECT = 0, NMG_BC_SLIP = 1, NMG_BC_OPEN = 2 };

/* Uniform Cartesian grid (paper Sec. 2, partition of the domain).  dim is 1
 * or 2; in 1D ny must be 1 and every face length |e| is 1; in 2D the faces
 * normal to x have length (y1-y0)/ny and those normal to y (x1-x0)/nx.
 * nx (and ny in 2D) must be divisible by 2^n_levels. */
typedef struct {
    int dim, nx, ny;
    double x0, x1, y0, y1;
} nmg_grid;

/* Boundary condition of one side (Remark on boundary conditions, Sec. 2.1).
 * kind REFLECT: ghost depth = interior depth, normal velocity reversed.
 * kind SLIP: normal velocity zero.  kind OPEN: the regime follows the
 * interior cell's local Froude number; qn is the discharge per unit width
 * flowing INTO the domain (> 0), h the ghost depth (> 0), ut the tangential
 * velocity (the physical v on the W/E sides, u on S/N).  NaN = not
 * prescribed; an OPEN side needs qn or h. */
typedef struct {
    int kind;
    double h, qn, ut;
} nmg_side;

typedef struct {
    nmg_side side[4];        /* W, E, S, N (1D uses W and E) */
} nmg_bc;

/* Method parameters.  Paper values: g = 9.81, alpha = 3 (eq:NewtonREG),
 * fd_eps = 1e-8 (eq:NumerDiff), tau = 1 (eq:NewtonREG-12), h_eps = 1e-6
 * (dry-cell remark), eps_r = 0.03 (LLF wave speed at wet/dry fronts),
 * N_L = n_levels = 3, n_mg = 2 (1D) / 3 (2D) cycles per Newton step, one
 * BLU-SGS pre-smoothing sweep per step (Algorithm 1, Step 2.1).  nu1/nu2
 * are the pre/post block-SGS iterations of Algorithm 0; nu_coarse the SGS
 * iterations that stand for the coarsest-level solve.  dry_pin (0/1) holds
 * the momentum of exactly dry cells at zero in the step that wets them;
 * pos_theta (>= 0, < 1) limits the per-cell relaxation so that no step
 * removes more than that fraction of a cell's depth (0 = tau everywhere).
 * inner_fp32 (0/1) stores the multigrid hierarchy (blocks, right-hand
 * sides, corrections) in FP32 and runs the V-cycle in FP32, while residuals,
 * assembly arithmetic, the update, the threshold and the stop test stay FP64
 * (Newton then acts as iterative refinement).  gamma is the cycle index of
 * Algorithm 0 (1 = V-cycle, 2 = W-cycle); the finest level always makes a
 * single coarse-grid call.  eps_p > 0 turns on Step 1 of Algorithm 1 in
 * nmg_newton_mg_solve: the initial data averaged onto the coarsest mesh
 * (children averaged level by level in the order SW, SE, NW, NE), then on
 * each level l = N_L..1 symmetric BLU-SGS sweeps while sum ||R_{i,l}||_1 >=
 * eps_p 2^-l (at most init_max_sweeps sweeps), then injection into the
 * children; eps_p = 0 starts Newton from U0 (the paper's experiments use
 * eps_p = 0.2 unless stated otherwise, and its remark on the parameter
 * suggests about 1 % of the initial residual).  Batches require eps_p = 0. */
typedef struct {
    int flux;
    double g, alpha, fd_eps, tau, h_eps, eps_r;
    int n_levels, nu1, nu2, nu_coarse, n_mg;
    int blu_sweeps, max_newton;
    int dry_pin;
    double pos_theta;
    int inner_fp32;
    int gamma;
    double eps_p;
    int init_max_sweeps;
} nmg_params;

/* Solve statistics (host memory).  res_hist (optional, host) receives the
 * sum of ||R_i||_1 at each Newton step, up to hist_cap entries. */
typedef struct {
    int newton_steps;        /* number of multigrid updates performed */
    int status;
    int n_pinned;            /* isolated cells at the returned state */
    double res_l1;           /* sum_i ||R_i||_1 of the returned state */
    double *res_hist;
    int hist_cap;
    int init_sweeps;         /* Step 1 BLU-SGS sweeps over all coarse levels */
    int init_level_sweeps[16];   /* Step 1 BLU-SGS sweeps on level l (0 for l = 0 and
                                    beyond n_levels) */
} nmg_stats;

/* Create a context for one grid / BC / parameter set on HIP stream `stream`
 * (hipStream_t, may be NULL for the null stream).  Allocates the
 * hierarchy.  Errors: EINVAL (inconsistent grid, BC or params), ENOMEM,
 * EHIP.
 *
 * Launch-structure switches, read from the environment here (and by
 * nmg_batch_create); none changes a bit of any result:
 *   NMG_COARSE_CELLS  levels of at most this many cells run inside one
 *                     single-workgroup kernel per cycle (default 1024; 0:
 *                     every level launched on its own);
 *   NMG_COARSE_REG    0 turns off register-resident runs on that kernel's
 *                     first level (default on);
 *   NMG_COARSE_SPLIT  0 gives every cell of the LDS-resident coarsest level
 *                     one lane in its runs of half sweeps (default: two
 *                     lanes per cell in 2D where the level has at most 128
 *                     cells per colour);
 *   NMG_FUSE          most half sweeps per launch on the launched coarse
 *                     levels: 3 (default), 2 or 1;
 *   NMG_BLU_LANES     lanes per cell of every BLU-SGS half sweep (Step 1 and
 *                     Step 2.1): 1, 4 (one per evaluation of the forward
 *                     differences) or 16 (one per face and evaluation, 2D;
 *                     4 in 1D); default: 16 in 2D on meshes of at most 2^14
 *                     cells per colour, 4 up to 2^16, else 1.
 *   NMG_STEP1_GRAPH   0: enqueue every Step 1 launch from the host; default
 *                     1: runs of 64 Step 1 sweeps on a level are captured
 *                     once per context as a HIP graph (on a stream of the
 *                     context's own) and replayed on the context's stream
 *                     (if capture or instantiation fails, the context
 *                     enqueues the launches one by one instead). */
int nmg_create(const nmg_grid *grid, const nmg_bc *bc, const nmg_params *params,
               void *stream, nmg_ctx **out);
void nmg_destroy(nmg_ctx *ctx);
const char *nmg_last_error(const nmg_ctx *ctx);

/* Local residuals R_i (eq:Res: sum over the cell's faces of |e| times the
 * edge term of eq:totalFlux) of state U over bed z.  R_out (device, nullable)
 * receives R in the cell-vector layout; res_l1_host (host, nullable) the sum
 * over cells of ||R_i||_1 (synchronizes the stream). */
int nmg_residual(nmg_ctx *ctx, const double *z, const double *U, double *R_out,
                 double *res_l1_host);

/* nmg_residual for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * no context, no allocation, no synchronization.  grid, bc and params are
 * validated as by nmg_create (n_levels must still divide the grid; nothing
 * else of params but the physics is used); z, U, R_out (nullable) as in
 * nmg_residual; res_l1 (DEVICE pointer, nullable) receives sum_i ||R_i||_1,
 * summed in the same order as nmg_residual's.  Enqueued on `stream`
 * (hipStream_t, NULL = null stream) of the current device.  The norm's block
 * partial sums go to a fixed device array of the library (2 MiB per GPU, kept
 * until the process ends), which limits the grid to nx * ny <= 2^26 cells;
 * larger grids return NMG_EINVAL, as do invalid arguments.  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (on different
 * streams, or from several threads) race.  NMG_EHIP if a launch fails. */
int nmg_residual_noalloc(const nmg_grid *grid, const nmg_bc *bc, const nmg_params *params,
                         void *stream, const double *z, const double *U, double *R_out,
                         double *res_l1);

/* Assembly of the level-0 Newton system eq:MatrixForm at state U: right-hand
 * side -R and blocks A_ii = alpha ||R_i||_1 I + sum_e |e| dF/dU_i,
 * A_ij = |e| dF/dU_j by forward differences (eq:NumerDiff, ghosts
 * re-evaluated on boundary faces), with isolated cells pinned, then the
 * Galerkin coarse levels (eq:ProjectAR, left).  The system stays in the
 * context for nmg_mg_vcycle.  R_out / res_l1_host as in nmg_residual. */
int nmg_assemble_residual_jacobian(nmg_ctx *ctx, const double *z, const double *U,
                                   double *R_out, double *res_l1_host);

/* n_cycles multigrid cycles (Algorithm 0 with the context's gamma,
 * red-black block SGS smoother) on the system last assembled or loaded,
 * starting from and returning dU (device, cell-vector layout, in/out). */
int nmg_mg_vcycle(nmg_ctx *ctx, double *dU, int n_cycles);

/* `iters` red-black block SGS iterations (red, black, black, red half
 * sweeps) on level `level` of the current hierarchy with that level's
 * right-hand side; dU in/out in the cell-vector layout of that level. */
int nmg_sgs(nmg_ctx *ctx, int level, double *dU, int iters);

/* One symmetric BLU-SGS sweep (Algorithm 1, Step 2.1; red, black, black,
 * red) on U in place, with the dry threshold after every cell update. */
int nmg_blu_sweep(nmg_ctx *ctx, const double *z, double *U);

/* Newton multigrid solve (Algorithm 1, Steps 2-3) from U (in: U0, out: the
 * returned iterate).  Each step: BLU-SGS sweeps, assembly, stop test
 * sum ||R_i||_1 < tol (the returned U is then the tested state), n_mg
 * V-cycles from dU = 0, relaxed update and dry threshold.  Returns OK,
 * NOT_CONVERGED, ENONFINITE, EDIVERGED or an error.  stats (host) nullable.
 * With Step 1 (eps_p > 0) and NMG_STEP1_GRAPH on, the first solve on a
 * context also creates a capture stream and one HIP graph per coarse level
 * (kept, and freed by nmg_destroy); the host synchronizes with the
 * context's stream once per run of Step 1 sweeps. */
int nmg_newton_mg_solve(nmg_ctx *ctx, const double *z, double *U, double tol,
                        nmg_stats *stats);

/* Load a level-0 system (A in the block layout, b) into the context and
 * build the Galerkin coarse levels from it.  For testing the linear
 * multigrid on its own. */
int nmg_load_system(nmg_ctx *ctx, const double *A0, const double *b0);

/* Copy level `level`'s blocks (nullable) and right-hand side (nullable) out
 * in the block / cell-vector layouts of that level (nx >> level,
 * ny >> level in 2D).  Coarse right-hand sides are those of the last cycle. */
int nmg_get_system(nmg_ctx *ctx, int level, double *A, double *b);

/* ---- Sensitivities of the steady state ------------------------------------
 * At a steady state R(U, z) = 0 an objective J(U, z) has the bed gradient
 * dJ/dz = dJ/dz|_U - (dR/dz)^T lambda, with (dR/dU)^T lambda = (dJ/dU)^T and
 * dR/dU the Newton matrix of eq:MatrixForm at (z, U) (the linearization the
 * solver uses, pinned rows included). */

/* Adjoint solve: assembles the Newton matrix at (z, U), transposes it block
 * by block (the transpose's block at cell i towards j is the transpose of
 * the block at j towards i), builds its Galerkin levels (which are the
 * transposes of the original's) and solves A^T lambda = g from the given
 * lambda (in/out, cell-vector layout) with multigrid cycles of the context's
 * kind: krylov = 0 iterates the cycles until ||g - A^T lambda||_1 <=
 * tol ||g - A^T lambda_in||_1; krylov = m > 0 (FP64 contexts, m <= 200)
 * accelerates them with GMRES(m), one cycle from zero being the right
 * preconditioner, until the 2-norm residual falls by tol.  At most
 * max_cycles cycles.  cycles_host and rel_res_host (nullable) receive the
 * number of cycles and the final l1 relative residual.  The transposed
 * system stays in the context (nmg_get_system shows it).  Synchronizes. */
int nmg_adjoint_solve(nmg_ctx *ctx, const double *z, const double *U, const double *g,
                      double *lambda, double tol, int max_cycles, int krylov, int *cycles_host,
                      double *rel_res_host);

/* out[ny][nx] = (dR/dz)^T lambda at (z, U): forward differences of the edge
 * terms in the bed with the absolute step fd_eps, face by face as the
 * Jacobian assembly differentiates in U (a boundary face's ghost carries the
 * raised bed), rows pinned as in the Newton matrix (isolated cell: zero row;
 * exactly dry cell with dry_pin: zero momentum rows).  out_j sums
 * lambda_j . dR_j/dz_j, then lambda_i . dR_i/dz_j over j's neighbours in W,
 * E, S, N order.  Stream-ordered, no synchronization. */
int nmg_bed_vjp(nmg_ctx *ctx, const double *z, const double *U, const double *lambda,
                double *out);

/* Measurement hooks.  With enable = 1 the library records a pair of
 * hipEvents on its stream around each run of full finest-level block SGS
 * half sweeps (ones that read every neighbour block) launched back to back
 * within one smoothing call, for at most `cap` (<= 2^20) runs; the events
 * are created here, so recording adds no allocation to the solve, and
 * enabling again drops earlier records.  enable = 0 stops recording.
 * nmg_timing_read synchronizes the stream and returns, over the recorded
 * runs, the summed milliseconds, the number of launches and the number of
 * cell updates they performed. */
int nmg_timing_enable(nmg_ctx *ctx, int enable, int cap);
int nmg_timing_read(nmg_ctx *ctx, double *sgs_ms_host, int *sgs_launches_host,
                    long long *sgs_cells_host);

/* Phases of nmg_newton_mg_solve (Algorithm 1).  STEP1: the dry threshold of
 * U0 and Step 1; BLU: the Step 2.1 sweeps (and the copy of the iterate kept
 * for a non-finite step); ASSEMBLY: isolation flags, residual and Jacobian of
 * level 0; GALERKIN: the coarse levels; NORM: the residual norm's reduction,
 * its transfer to the host and the stop test; CYCLES: the n_mg multigrid
 * cycles; UPDATE: the relaxed update and threshold; FINAL: the returned
 * state's residual norm and pinned-cell count. */
enum { NMG_PHASE_STEP1 = 0, NMG_PHASE_BLU, NMG_PHASE_ASSEMBLY, NMG_PHASE_GALERKIN,
       NMG_PHASE_NORM, NMG_PHASE_CYCLES, NMG_PHASE_UPDATE, NMG_PHASE_FINAL, NMG_NPHASES };

/* With timing enabled, nmg_newton_mg_solve also records one event on the
 * stream at each phase boundary (at most `cap` events, the same cap as
 * above).  nmg_timing_phases synchronizes the stream and returns in
 * ms_host[NMG_NPHASES] (host) the milliseconds between consecutive events
 * summed per phase over the recorded solves, i.e. the stream's wall time in
 * each phase, idle gaps (host round trips of the stop test) included;
 * marks_host (nullable) the number of events recorded. */
int nmg_timing_phases(nmg_ctx *ctx, double *ms_host, int *marks_host);

/* ---- Batches of independent problems --------------------------------------
 * A batch solves n independent steady problems (Algorithm 1 on each) of
 * possibly different grid sizes and boundary data but one parameter set, in
 * lockstep: every operation of the Newton step and of the multigrid cycle is
 * one launch over a work list of (instance, tile) items of all instances
 * still iterating, and the coarse part of each cycle runs one workgroup per
 * instance.  Every instance's iterates, statuses and step counts are those
 * of its own nmg_newton_mg_solve with the same grid, BC and parameters, bit
 * for bit; an instance leaves the lockstep when its own stop test ends it.
 * Requirements: all grids have the same dim, and each satisfies
 * nmg_create's rules with params->n_levels. */
typedef struct nmg_batch nmg_batch;

/* grids[n], bcs[n] (host arrays), one params for all instances, stream as in
 * nmg_create.  Allocates one hierarchy per instance plus the work lists.
 * Launch-structure switch read here (changes no bit of any result):
 * NMG_BATCH_PERSISTENT = k > 0 runs the batched half sweeps on a persistent
 * grid of k blocks per compute unit looping over the work list (default:
 * one block per work item). */
int nmg_batch_create(int n, const nmg_grid *grids, const nmg_bc *bcs,
                     const nmg_params *params, void *stream, nmg_batch **out);
void nmg_batch_destroy(nmg_batch *batch);
const char *nmg_batch_last_error(const nmg_batch *batch);

/* Tile-length autotuner of the batched block SGS half sweep: for every
 * level launched on its own (the coarse-kernel levels excepted), times
 * `reps` (1..1000) half sweeps with each tile length 64, 128, 256 and 512
 * cells on this batch's hierarchy and keeps the fastest.  Results do not
 * depend on the choice.  tiles_host (nullable, n_levels + 1 ints) receives
 * the chosen lengths.  Synchronizes the stream. */
int nmg_batch_autotune(nmg_batch *batch, int reps, int *tiles_host);

/* Newton multigrid solves of every instance: z[k], U[k] are device pointers
 * (the host arrays z, U hold n of them) with the layouts of
 * nmg_newton_mg_solve; U[k] in: U0, out: the returned iterate.  stats (host,
 * n entries, nullable) receives each instance's result as
 * nmg_newton_mg_solve would.  Returns NMG_OK if every instance converged,
 * NMG_NOT_CONVERGED if any did not (see stats), or an error. */
int nmg_batch_newton_mg_solve(nmg_batch *batch, const double *const *z, double *const *U,
                              double tol, nmg_stats *stats);

#ifdef __cplusplus
}
#endif
#endif /* NMG_H */
