/*
 * Plain FP64 CPU oracle for the Newton multigrid method of Wu & Tang,
 * "A Newton multigrid method for steady-state shallow water equations with
 * topography and dry areas" (arXiv:1608.06721).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path.  It
 * is loaded by the test-suite, by the smoke check and by the CPU-baseline leg
 * of the benchmark, and by nothing else.  The product path never calls it and
 * shares no source with it.
 *
 * Layouts (all row-major, x fastest):
 *   cell vectors   v[c][ny][nx]                  c < NC (2 in 1D, 3 in 2D)
 *   block matrices A[b][r][c][ny][nx]            b in (D, W, E, S, N); 1D has (D, W, E)
 * A[b][r][c] at cell i is d(row r of cell i's equation)/d(component c of the
 * unknown of the cell that block b points to): D = the cell itself, W/E/S/N =
 * its face neighbours.
 */
#ifndef NMG_ORACLE_H
#define NMG_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_REFLECT = 0, ORC_SLIP = 1, ORC_OPEN = 2 };
enum { ORC_HLL = 0, ORC_LLF = 1, ORC_HLLC = 2 };
enum { ORC_REDBLACK = 0, ORC_LEX = 1 };
enum { ORC_OK = 0, ORC_NOT_CONVERGED = 1, ORC_EINVAL = -1, ORC_ENONFINITE = -4,
       ORC_EDIVERGED = -5 };

typedef struct {
    int dim, nx, ny;                /* ny = 1 when dim = 1 */
    double x0, x1, y0, y1;
} orc_grid;

/* One side of the domain.  NaN means "not prescribed".
 * h: depth; qn: discharge per unit width flowing INTO the domain (> 0);
 * ut: tangential velocity (the physical v on W/E sides, u on S/N sides). */
typedef struct {
    int kind;
    double h, qn, ut;
} orc_side;

typedef struct {
    int flux;
    double g, alpha, fd_eps, tau, h_eps, eps_r;
    int n_levels;                   /* N_L: number of coarse levels */
    int nu1, nu2, nu_coarse, n_mg;
    int blu_sweeps, max_newton, order;
    int dry_pin;                    /* hold the momentum of exactly dry cells at 0 */
    double pos_theta;               /* positivity limit of the per-cell relaxation (0 = off) */
    int inner_fp32;                 /* V-cycles in FP32 (Newton residual and update in FP64) */
    int gamma;                      /* cycle index: 1 = V-cycle, 2 = W-cycle */
    double eps_p;                   /* Step 1 tolerance; <= 0: start Newton from U0 directly */
    int init_max_sweeps;            /* Step 1: at most this many BLU-SGS sweeps per level */
} orc_params;

typedef struct {
    int newton_steps, status, n_pinned;
    double res_l1;
    double *res_hist;
    int hist_cap;
    int init_sweeps;                /* Step 1 BLU-SGS sweeps over all levels */
} orc_stats;

/* --- pieces exposed for unit tests ------------------------------------ */
void orc_num_flux(int flux, int nc, int axis, double g, double eps_r,
                  double hL, double uL, double vL, double hR, double uR, double vR,
                  double out[3]);
void orc_phys_flux(int nc, int axis, double g, double h, double u, double v, double out[3]);
/* ghost state (h, u, v) for interior state (h, u, v) on side f (0 W, 1 E, 2 S, 3 N) */
void orc_ghost(const orc_side *bc, int f, double g, double h_eps,
               double h, double u, double v, double out[3]);
double orc_inflow_celerity(double K, double gq);
void orc_solve_block(int nc, const double *D /* row-major nc*nc */, const double *r, double *x);

/* --- discretization ----------------------------------------------------- */
/* Threads of the oracle's independent per-cell loops (default 1; results do
 * not depend on it). */
void orc_set_threads(int n);
int orc_get_threads(void);

int orc_residual(const orc_grid *gr, const orc_side bc[4], const orc_params *p,
                 const double *z, const double *U, double *R, double *res_l1);
int orc_isolated(const orc_grid *gr, const orc_side bc[4], const orc_params *p,
                 const double *z, const double *U, unsigned char *iso);
int orc_assemble(const orc_grid *gr, const orc_side bc[4], const orc_params *p,
                 const double *z, const double *U, double *A, double *b, double *res_l1);

/* --- linear multigrid pieces (dim, nx, ny of the level they act on) ---- */
void orc_galerkin(int dim, int nx, int ny, const double *Af, double *Ac);
void orc_sgs_half(int dim, int nx, int ny, const double *A, const double *b, double *x,
                  int color);
void orc_sgs(int dim, int nx, int ny, const double *A, const double *b, double *x,
             int iters, int order);
void orc_lin_residual(int dim, int nx, int ny, const double *A, const double *b,
                      const double *x, double *r);
void orc_restrict(int dim, int nx, int ny, const double *A, const double *b,
                  const double *x, double *bc);
void orc_prolong(int dim, int nx, int ny, const double *xc, double *x);
/* n_cycles V-cycles on the hierarchy built by Galerkin from A0; x in/out.
 * With p->inner_fp32 the hierarchy and the cycles are FP32 (A0, b0, x
 * rounded on entry, x widened on return). */
int orc_vcycles(int dim, int nx, int ny, const orc_params *p, const double *A0,
                const double *b0, double *x, int n_cycles);

/* --- nonlinear driver --------------------------------------------------- */
int orc_blu_sweep(const orc_grid *gr, const orc_side bc[4], const orc_params *p,
                  const double *z, double *U);
void orc_threshold(const orc_grid *gr, const orc_params *p, double *U);
int orc_newton_solve(const orc_grid *gr, const orc_side bc[4], const orc_params *p,
                     const double *z, double *U, double tol, orc_stats *st);

/* Algorithm 1, Step 1: nested initial guess of U (in: the initial data on
 * level 0, out: Newton's initial guess); sweeps[l] (nullable, n_levels + 1
 * entries) receives the BLU-SGS sweeps done on level l. */
int orc_nested_init(const orc_grid *gr, const orc_side bc[4], const orc_params *p,
                    const double *z, double *U, int *sweeps);

/* --- sensitivities (adjoint of the steady state) ------------------------- */
/* Exact block transpose: At's block at cell i towards neighbour j is A's
 * block at j towards i, transposed; diagonal blocks transposed in place. */
void orc_transpose_blocks(int dim, int nx, int ny, const double *A, double *At);
/* out = (dR/dz)^T lam by forward differences of the edge terms in the bed,
 * rows pinned as in orc_assemble (see the definition). */
int orc_bed_vjp(const orc_grid *gr, const orc_side bc[4], const orc_params *p,
                const double *z, const double *U, const double *lam, double *out);

#ifdef __cplusplus
}
#endif
#endif
