/*
 * Plain FP64 CPU oracle of the Newton multigrid method (Wu & Tang,
 * arXiv:1608.06721).  TEST INFRASTRUCTURE ONLY: it is what the GPU path is
 * checked against, and only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load it.
 *
 * Written to be read against the paper, not to be fast: one cell at a time,
 * scalar loops, no blocking, no fusion.  Every floating-point expression is
 * written in the order stated in the comments (the order is part of the
 * definition, because the GPU path is required to reproduce it bit for bit).
 * Build with -O2 -ffp-contract=off and without fast-math.
 *
 * Section references are to the paper: Sec. 2.1 (well-balanced finite volume
 * discretization, eq:DSeqs, eq:totalFlux, Remark on fluxes, Remark on
 * boundary conditions), Sec. 2.2 (Newton, eq:NumerDiff, eq:NewtonREG,
 * eq:NewtonREG-12), Sec. 2.3 (eq:MatrixForm, eq:ProjectAR, eq:correction,
 * Algorithm 0), Sec. 2.4 (Algorithm 1 and the dry-cell remark).
 *
 * Parity unpinned: the positivity limit of the relaxed update (pos_theta)
 * and the cap on Step 1 sweeps per level (init_max_sweeps) are parameters
 * of this implementation that the paper does not have; their definitions
 * are checked (tests), but no value in the paper pins them.
 */
#include "nmg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Threads of the per-cell loops whose iterations are independent: cells of
 * one colour in a red-black half sweep, and loops that only read the state
 * they do not write (residual, assembly, restriction, Galerkin sums,
 * updates).  One by default; the lexicographic sweeps and every sum over
 * cells stay sequential in cell order, so results do not depend on it. */
static int orc_threads = 1;

void orc_set_threads(int n) { orc_threads = n > 0 ? n : 1; }
int orc_get_threads(void) { return orc_threads; }

#define ORC_PARALLEL_FOR _Pragma("omp parallel for schedule(static) num_threads(orc_threads) if (orc_threads > 1)")

enum { FW = 0, FE = 1, FS = 2, FN = 3 };

/* max/min written as comparisons so that a NaN operand in the second place
 * propagates (max(0, NaN) = NaN). */
static double dmax(double a, double b) { return a > b ? a : b; }
static double dmin(double a, double b) { return a < b ? a : b; }

/* ------------------------------------------------------------------------ */
/* Physical flux F_n(U) of Sec. 1 along coordinate axis `axis` (0 = x, 1 = y)
 * for the state U = (h, h u, h v):  (h u_n, h u_n u + g/2 h^2 n_x,
 * h u_n v + g/2 h^2 n_y).  m = h * u_n, p = 0.5 * g * h * h. */
void orc_phys_flux(int nc, int axis, double g, double h, double u, double v, double out[3])
{
    double un = (axis == 0) ? u : v;
    double m = h * un;
    double p = 0.5 * g * h * h;
    out[0] = m;
    out[1] = (axis == 0) ? m * u + p : m * u;
    if (nc == 3) out[2] = (axis == 1) ? m * v + p : m * v;
}

/* Numerical flux across a face whose normal is the +axis direction, between
 * the reconstructed left state (hL, uL, vL) and right state (hR, uR, vR)
 * (Remark on numerical fluxes, Sec. 2.1).  Velocities are the cell
 * velocities even where the reconstructed depth is zero. */
void orc_num_flux(int flux, int nc, int axis, double g, double eps_r,
                  double hL, double uL, double vL, double hR, double uR, double vR,
                  double out[3])
{
    double FL[3] = {0, 0, 0}, FR[3] = {0, 0, 0};
    double UL[3] = {0, 0, 0}, UR[3] = {0, 0, 0};
    orc_phys_flux(nc, axis, g, hL, uL, vL, FL);
    orc_phys_flux(nc, axis, g, hR, uR, vR, FR);
    UL[0] = hL; UL[1] = hL * uL; UL[2] = hL * vL;
    UR[0] = hR; UR[1] = hR * uR; UR[2] = hR * vR;
    double unL = (axis == 0) ? uL : vL;
    double unR = (axis == 0) ? uR : vR;
    double cL = sqrt(g * hL), cR = sqrt(g * hR);

    if (flux == ORC_LLF) {
        /* eq:LLFflux with the wet/dry-enlarged wave speed (eps_r term). */
        double s = dmax(fabs(unL) + cL, fabs(unR) + cR) + eps_r * sqrt(g * dmax(hL, hR));
        for (int k = 0; k < nc; ++k)
            out[k] = 0.5 * ((FL[k] + FR[k]) - s * (UR[k] - UL[k]));
        return;
    }
    /* eq:HLLflux with the two-rarefaction star estimates u_*, h_*; HLLC
     * adds the contact wave s_M for the tangential momentum below. */
    double us = ((unL + unR) * 0.5 + cL) - cR;
    double a = (cL + cR) + (unL - unR) * 0.5;
    double hs = (a * a) / (4.0 * g);
    double cs = sqrt(g * hs);
    double sL = (hL == 0.0) ? unR - 2.0 * cR : dmin(unL - cL, us - cs);
    double sR = (hR == 0.0) ? unL + 2.0 * cL : dmax(unR + cR, us + cs);
    if (sL >= 0.0) {
        for (int k = 0; k < nc; ++k) out[k] = FL[k];
    } else if (sR <= 0.0) {
        for (int k = 0; k < nc; ++k) out[k] = FR[k];
    } else {
        for (int k = 0; k < nc; ++k)
            out[k] = ((sR * FL[k] - sL * FR[k]) + (sL * sR) * (UR[k] - UL[k])) / (sR - sL);
        if (flux == ORC_HLLC && nc == 3) {
            /* HLLC (Remark on numerical fluxes): the tangential momentum flux
             * is the upwind tangential velocity, chosen by the sign of the
             * contact speed s_M, times the HLL mass flux.  s_M's 0/0 (both
             * sides dry) is taken as 0. */
            double num = (sL * hR) * (unR - sR) - (sR * hL) * (unL - sL);
            double den = hR * (unR - sR) - hL * (unL - sL);
            double sM = (den != 0.0) ? num / den : 0.0;
            double utL = (axis == 0) ? vL : uL, utR = (axis == 0) ? vR : uR;
            double ut = (sM >= 0.0) ? utL : utR;
            out[2 - axis] = ut * out[0];
        }
    }
}

/* Positive root c of 2 c^3 - K c^2 - gq = 0 (gq > 0).  With c = sqrt(g h_g)
 * this is the subcritical-inflow ghost depth: the outgoing invariant
 * u_n + 2 sqrt(g h) is carried from the interior and h_g u_n,g = -q.  Newton
 * from an upper bound of the root; the iterates decrease monotonically, and
 * the loop stops at the first step that does not decrease c. */
double orc_inflow_celerity(double K, double gq)
{
    double c = dmax(K, 0.0) + dmax(1.0, gq);
    for (int it = 0; it < 100; ++it) {
        double f = (2.0 * c - K) * c * c - gq;
        double fp = (6.0 * c - 2.0 * K) * c;
        double cn = c - f / fp;
        if (!(cn < c)) break;
        c = cn;
    }
    return c;
}

/* Ghost state of the Remark on boundary conditions (Sec. 2.1).  `f` is the
 * side (W, E, S, N); the outward normal is -x, +x, -y, +y.  Input and output
 * are (h, u, v) with u, v the physical velocity components. */
void orc_ghost(const orc_side *bc, int f, double g, double h_eps,
               double h, double u, double v, double out[3])
{
    int axis = (f == FW || f == FE) ? 0 : 1;
    double sgn = (f == FW || f == FS) ? -1.0 : 1.0;
    double un_in = sgn * (axis == 0 ? u : v);   /* outward normal velocity */
    double ut_in = (axis == 0) ? v : u;         /* tangential component */
    double hg, ung, utg;

    if (bc->kind == ORC_REFLECT) {
        hg = h; ung = -un_in; utg = ut_in;
    } else if (bc->kind == ORC_SLIP) {
        hg = h; ung = 0.0; utg = ut_in;
    } else {
        /* Open side: regime from the interior cell's local Froude number. */
        int super = (h > h_eps) && (u * u + v * v >= g * h);
        int outflow = un_in >= 0.0;
        int hasq = !isnan(bc->qn), hash = !isnan(bc->h), hast = !isnan(bc->ut);
        if (super && outflow) {                      /* supercritical outflow */
            hg = h; ung = un_in; utg = ut_in;
        } else if (super && hasq && hash && hast) {  /* supercritical inflow */
            hg = bc->h; ung = -bc->qn / bc->h; utg = bc->ut;
        } else if (hasq && (!hash || !outflow)) {    /* subcritical, discharge given */
            double K = un_in + 2.0 * sqrt(g * h);
            double c = orc_inflow_celerity(K, g * bc->qn);
            hg = c * c / g;
            ung = -bc->qn / hg;
            utg = hast ? bc->ut : 0.0;
        } else {                                     /* subcritical, depth given */
            hg = bc->h;
            ung = (un_in + 2.0 * sqrt(g * h)) - 2.0 * sqrt(g * hg);
            utg = ut_in;
        }
    }
    out[0] = hg;
    if (axis == 0) { out[1] = sgn * ung; out[2] = utg; }
    else           { out[1] = utg;       out[2] = sgn * ung; }
}

/* ------------------------------------------------------------------------ */
/* Problem description shared by the discretization routines. */
typedef struct {
    const orc_grid *gr;
    const orc_side *bc;
    const orc_params *p;
    const double *z;
    int nc, nf, N;
    double elen[4];           /* |e| of the W, E, S, N faces */
} prob;

typedef struct { double h, u, v, z; } side_t;   /* one side of a face */

static int setup(prob *P, const orc_grid *gr, const orc_side *bc, const orc_params *p,
                 const double *z)
{
    if (gr->dim != 1 && gr->dim != 2) return ORC_EINVAL;
    if (gr->nx < 1 || gr->ny < 1 || (gr->dim == 1 && gr->ny != 1)) return ORC_EINVAL;
    P->gr = gr; P->bc = bc; P->p = p; P->z = z;
    P->nc = gr->dim == 1 ? 2 : 3;
    P->nf = gr->dim == 1 ? 2 : 4;
    P->N = gr->nx * gr->ny;
    if (gr->dim == 1) {
        P->elen[0] = P->elen[1] = P->elen[2] = P->elen[3] = 1.0;
    } else {
        double dx = (gr->x1 - gr->x0) / gr->nx, dy = (gr->y1 - gr->y0) / gr->ny;
        P->elen[FW] = P->elen[FE] = dy;
        P->elen[FS] = P->elen[FN] = dx;
    }
    return ORC_OK;
}

/* Cell velocity: hu/h where the cell is wet (h > h_eps), otherwise 0. */
static double vel(double h, double m, double h_eps) { return h > h_eps ? m / h : 0.0; }

static side_t cell_side(const prob *P, const double *Uc, double z)
{
    side_t s;
    s.h = Uc[0];
    s.u = vel(Uc[0], Uc[1], P->p->h_eps);
    s.v = (P->nc == 3) ? vel(Uc[0], Uc[2], P->p->h_eps) : 0.0;
    s.z = z;
    return s;
}

static side_t ghost_side(const prob *P, int f, side_t in)
{
    double o[3];
    orc_ghost(&P->bc[f], f, P->p->g, P->p->h_eps, in.h, in.u, in.v, o);
    side_t s = {o[0], o[1], o[2], in.z};   /* ghost bed = interior bed */
    return s;
}

/* Reconstructed depths on the two sides of a face (hydrostatic
 * reconstruction, Sec. 2.1): h_pm = max(0, h + z - max(zL, zR)). */
static void recon(side_t L, side_t R, double *hL, double *hR)
{
    double zM = dmax(L.z, R.z);
    *hL = dmax(0.0, L.h + L.z - zM);
    *hR = dmax(0.0, R.h + R.z - zM);
}

/* Edge term of eq:totalFlux for the cell on side `own` of its face f, the
 * other side being `oth`.  The numerical flux of a face is evaluated once in
 * the +axis orientation (left = lower coordinate), so the scheme is exactly
 * conservative; the cell on the left takes  F - S(h_left), the cell on the
 * right takes -F + S(h_right), S carrying g/2 h^2 in the normal momentum. */
static void edge_term(const prob *P, int f, side_t own, side_t oth, double T[3])
{
    int axis = (f == FW || f == FE) ? 0 : 1;
    int own_left = (f == FE || f == FN);
    side_t L = own_left ? own : oth;
    side_t R = own_left ? oth : own;
    double hL, hR, F[3] = {0, 0, 0};
    recon(L, R, &hL, &hR);
    orc_num_flux(P->p->flux, P->nc, axis, P->p->g, P->p->eps_r, hL, L.u, L.v, hR, R.u, R.v, F);
    double ho = own_left ? hL : hR;
    double po = 0.5 * P->p->g * ho * ho;
    for (int k = 0; k < P->nc; ++k) T[k] = own_left ? F[k] : -F[k];
    if (own_left) T[1 + axis] = F[1 + axis] - po;
    else          T[1 + axis] = -F[1 + axis] + po;
}

/* Neighbour of (i, j) across face f, or 0 on the domain boundary. */
static int nbr(int dim, int nx, int ny, int i, int j, int f, int *ni, int *nj)
{
    *ni = i; *nj = j;
    if (f == FW) { if (i == 0) return 0; *ni = i - 1; return 1; }
    if (f == FE) { if (i == nx - 1) return 0; *ni = i + 1; return 1; }
    if (dim == 1) return 0;
    if (f == FS) { if (j == 0) return 0; *nj = j - 1; return 1; }
    if (j == ny - 1) return 0;
    *nj = j + 1;
    return 1;
}

static void load_cell(const prob *P, const double *U, int idx, double *Uc)
{
    for (int k = 0; k < P->nc; ++k) Uc[k] = U[k * P->N + idx];
}

/* Edge term of cell (i, j) on face f with the cell's state Ui and the
 * neighbour's state Uj (ignored on the boundary, where the ghost is built
 * from Ui). */
static void cell_edge(const prob *P, int i, int j, int f, const double *Ui, const double *Uj,
                      double T[3])
{
    int nx = P->gr->nx, ni, nj;
    side_t own = cell_side(P, Ui, P->z[j * nx + i]);
    side_t oth;
    if (nbr(P->gr->dim, nx, P->gr->ny, i, j, f, &ni, &nj))
        oth = cell_side(P, Uj, P->z[nj * nx + ni]);
    else
        oth = ghost_side(P, f, own);
    edge_term(P, f, own, oth, T);
}

/* Local residual R_i = sum over faces (W, E, S, N order) of |e| T (eq:Res). */
static void cell_residual(const prob *P, const double *U, int i, int j, double *Rc)
{
    int nx = P->gr->nx, ni, nj;
    double Ui[3], Uj[3] = {0, 0, 0}, T[3];
    load_cell(P, U, j * nx + i, Ui);
    for (int k = 0; k < P->nc; ++k) Rc[k] = 0.0;
    for (int f = 0; f < P->nf; ++f) {
        if (nbr(P->gr->dim, nx, P->gr->ny, i, j, f, &ni, &nj)) load_cell(P, U, nj * nx + ni, Uj);
        cell_edge(P, i, j, f, Ui, Uj, T);
        for (int k = 0; k < P->nc; ++k) Rc[k] = Rc[k] + P->elen[f] * T[k];
    }
}

static double l1(int nc, const double *Rc)
{
    double s = fabs(Rc[0]) + fabs(Rc[1]);
    if (nc == 3) s = s + fabs(Rc[2]);
    return s;
}

int orc_residual(const orc_grid *gr, const orc_side bc[4], const orc_params *p,
                 const double *z, const double *U, double *R, double *res_l1)
{
    prob P;
    if (setup(&P, gr, bc, p, z)) return ORC_EINVAL;
    double *nrm = (double *)malloc(sizeof(double) * (size_t)P.N);
    if (!nrm) return ORC_EINVAL;
    ORC_PARALLEL_FOR
    for (int j = 0; j < gr->ny; ++j)
        for (int i = 0; i < gr->nx; ++i) {
            double Rc[3];
            cell_residual(&P, U, i, j, Rc);
            for (int k = 0; k < P.nc; ++k) if (R) R[k * P.N + j * gr->nx + i] = Rc[k];
            nrm[j * gr->nx + i] = l1(P.nc, Rc);
        }
    double tot = 0.0;
    for (int idx = 0; idx < P.N; ++idx) tot = tot + nrm[idx];
    free(nrm);
    if (res_l1) *res_l1 = tot;
    return ORC_OK;
}

/* A cell is isolated when every one of its faces has zero reconstructed
 * depth on both sides: nothing flows in or out and nothing presses on it, so
 * R_i = 0 and its diagonal block is singular.  Such a cell keeps dU_i = 0. */
static int cell_isolated(const prob *P, const double *U, int i, int j)
{
    int nx = P->gr->nx, ni, nj;
    double Ui[3], Uj[3];
    load_cell(P, U, j * nx + i, Ui);
    side_t own = cell_side(P, Ui, P->z[j * nx + i]);
    for (int f = 0; f < P->nf; ++f) {
        side_t oth;
        if (nbr(P->gr->dim, nx, P->gr->ny, i, j, f, &ni, &nj)) {
            load_cell(P, U, nj * nx + ni, Uj);
            oth = cell_side(P, Uj, P->z[nj * nx + ni]);
        } else {
            oth = ghost_side(P, f, own);
        }
        double hL, hR;
        recon(own, oth, &hL, &hR);
        if (hL != 0.0 || hR != 0.0) return 0;
    }
    return 1;
}

int orc_isolated(const orc_grid *gr, const orc_side bc[4], const orc_params *p,
                 const double *z, const double *U, unsigned char *iso)
{
    prob P;
    if (setup(&P, gr, bc, p, z)) return ORC_EINVAL;
    ORC_PARALLEL_FOR
    for (int j = 0; j < gr->ny; ++j)
        for (int i = 0; i < gr->nx; ++i) iso[j * gr->nx + i] = (unsigned char)cell_isolated(&P, U, i, j);
    return ORC_OK;
}

#define AIDX(P, b, r, c, idx) ((((size_t)(b) * (P)->nc + (r)) * (P)->nc + (c)) * (P)->N + (idx))

/* Cell residual and forward-difference diagonal block dR_i/dU_i
 * (eq:NumerDiff, with the ghost re-evaluated from the perturbed state on
 * boundary faces); optionally the off-diagonal blocks dR_i/dU_j. */
static void cell_jacobian(const prob *P, const double *U, int i, int j, double *Rc,
                          double Dm[3][3], double Off[4][3][3])
{
    int nx = P->gr->nx, nc = P->nc, ni, nj;
    double eps = P->p->fd_eps;
    double Ui[3], Uj[3] = {0, 0, 0}, T0[3], Tk[3], Up[3];
    load_cell(P, U, j * nx + i, Ui);
    for (int r = 0; r < nc; ++r) {
        Rc[r] = 0.0;
        for (int c = 0; c < nc; ++c) Dm[r][c] = 0.0;
    }
    if (Off) memset(Off, 0, sizeof(double) * 4 * 9);
    for (int f = 0; f < P->nf; ++f) {
        double e = P->elen[f];
        int inner = nbr(P->gr->dim, nx, P->gr->ny, i, j, f, &ni, &nj);
        if (inner) load_cell(P, U, nj * nx + ni, Uj);
        cell_edge(P, i, j, f, Ui, Uj, T0);
        for (int r = 0; r < nc; ++r) Rc[r] = Rc[r] + e * T0[r];
        for (int k = 0; k < nc; ++k) {          /* perturb own component k */
            memcpy(Up, Ui, sizeof Up);
            Up[k] = Up[k] + eps;
            cell_edge(P, i, j, f, Up, Uj, Tk);
            for (int r = 0; r < nc; ++r) Dm[r][k] = Dm[r][k] + e * ((Tk[r] - T0[r]) / eps);
        }
        if (inner && Off) {
            for (int k = 0; k < nc; ++k) {      /* perturb neighbour component k */
                memcpy(Up, Uj, sizeof Up);
                Up[k] = Up[k] + eps;
                cell_edge(P, i, j, f, Ui, Up, Tk);
                for (int r = 0; r < nc; ++r) Off[f][r][k] = e * ((Tk[r] - T0[r]) / eps);
            }
        }
    }
}

/* A cell that is exactly dry (h = 0) has zero velocity, so its momentum
 * columns vanish and its momentum rows carry only the regularization, which
 * scales like the small residual of a freshly wetting cell.  With the
 * dry-cell pin its momentum unknowns are held at zero for this step: their
 * rows become the mass diagonal entry times the identity with a zero right-
 * hand side, so the cell can take on water (mass row untouched) but starts
 * at rest. */
static void dry_momentum_pin(int nc, double *Rc, double Dm[3][3], double Off[4][3][3])
{
    for (int r = 1; r < nc; ++r) {
        for (int c = 0; c < nc; ++c) {
            Dm[r][c] = 0.0;
            if (Off)
                for (int f = 0; f < 4; ++f) Off[f][r][c] = 0.0;
        }
        Dm[r][r] = Dm[0][0];
        Rc[r] = 0.0;
    }
}

/* Assembly of eq:MatrixForm at level 0: b = -R and the blocks
 * A_ii = alpha ||R_i||_1 I + sum_e |e| dF/dU_i,  A_ij = |e| dF/dU_j
 * (eq:NewtonREG).  Isolated cells are pinned: zero diagonal block, zero row,
 * zero right-hand side, and zero column in their neighbours' rows. */
int orc_assemble(const orc_grid *gr, const orc_side bc[4], const orc_params *p,
                 const double *z, const double *U, double *A, double *b, double *res_l1)
{
    prob P;
    if (setup(&P, gr, bc, p, z)) return ORC_EINVAL;
    int nx = gr->nx, ny = gr->ny, nc = P.nc, nb = P.nf + 1;
    unsigned char *iso = (unsigned char *)malloc((size_t)P.N);
    double *nrms = (double *)malloc(sizeof(double) * (size_t)P.N);
    if (!iso || !nrms) { free(iso); free(nrms); return ORC_EINVAL; }
    orc_isolated(gr, bc, p, z, U, iso);
    ORC_PARALLEL_FOR
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            int idx = j * nx + i, ni, nj;
            double Rc[3], Dm[3][3], Off[4][3][3];
            cell_jacobian(&P, U, i, j, Rc, Dm, Off);
            double nrm = l1(nc, Rc);
            nrms[idx] = nrm;
            for (int r = 0; r < nc; ++r) Dm[r][r] = Dm[r][r] + p->alpha * nrm;
            if (iso[idx]) {
                memset(Dm, 0, sizeof Dm);
                memset(Off, 0, sizeof Off);
            } else if (p->dry_pin && U[idx] == 0.0) {
                dry_momentum_pin(nc, Rc, Dm, Off);
            }
            for (int f = 0; f < P.nf; ++f)
                if (nbr(gr->dim, nx, ny, i, j, f, &ni, &nj) && iso[nj * nx + ni])
                    memset(Off[f], 0, sizeof Off[f]);
            for (int r = 0; r < nc; ++r) {
                b[r * P.N + idx] = iso[idx] ? 0.0 : -Rc[r];
                for (int c = 0; c < nc; ++c) {
                    A[AIDX(&P, 0, r, c, idx)] = Dm[r][c];
                    for (int f = 0; f < P.nf; ++f) A[AIDX(&P, f + 1, r, c, idx)] = Off[f][r][c];
                }
            }
            (void)nb;
        }
    double tot = 0.0;
    for (int idx = 0; idx < P.N; ++idx) tot = tot + nrms[idx];
    free(iso);
    free(nrms);
    if (res_l1) *res_l1 = tot;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Linear multigrid on one level: dims (dim, nx, ny), matrix A, vectors. */
typedef struct { int dim, nx, ny, nc, nf, N; } lvl;

static lvl mklvl(int dim, int nx, int ny)
{
    lvl L = {dim, nx, ny, dim == 1 ? 2 : 3, dim == 1 ? 2 : 4, nx * ny};
    return L;
}

#define LA(L, b, r, c, idx) ((((size_t)(b) * (L)->nc + (r)) * (L)->nc + (c)) * (L)->N + (idx))

/* Children of coarse cell (I, J) in the order SW, SE, NW, NE (1D: left,
 * right).  Returns the count. */
static int children(const lvl *Lf, int I, int J, int ci[4], int cj[4])
{
    if (Lf->dim == 1) {
        ci[0] = 2 * I; ci[1] = 2 * I + 1; cj[0] = cj[1] = 0;
        return 2;
    }
    ci[0] = 2 * I;     cj[0] = 2 * J;
    ci[1] = 2 * I + 1; cj[1] = 2 * J;
    ci[2] = 2 * I;     cj[2] = 2 * J + 1;
    ci[3] = 2 * I + 1; cj[3] = 2 * J + 1;
    return 4;
}

/* The linear multigrid in FP64 (suffix _d) and, for the FP32 inner
 * V-cycle, in FP32 (suffix _f). */
#define REAL double
#define MG(name) name##_d
#include "nmg_oracle_mg.inc"
#undef REAL
#undef MG
#define REAL float
#define MG(name) name##_f
#include "nmg_oracle_mg.inc"
#undef REAL
#undef MG

void orc_solve_block(int nc, const double *D, const double *r, double *x)
{
    solve_block_d(nc, D, r, x);
}

void orc_sgs_half(int dim, int nx, int ny, const double *A, const double *b, double *x, int color)
{
    sgs_half_d(dim, nx, ny, A, b, x, color);
}

void orc_sgs(int dim, int nx, int ny, const double *A, const double *b, double *x, int iters,
             int order)
{
    sgs_d(dim, nx, ny, A, b, x, iters, order);
}

void orc_lin_residual(int dim, int nx, int ny, const double *A, const double *b, const double *x,
                      double *r)
{
    lin_residual_d(dim, nx, ny, A, b, x, r);
}

void orc_restrict(int dim, int nx, int ny, const double *A, const double *b, const double *x,
                  double *bc)
{
    restrict__d(dim, nx, ny, A, b, x, bc);
}

void orc_prolong(int dim, int nx, int ny, const double *xc, double *x)
{
    prolong_d(dim, nx, ny, xc, x);
}

void orc_galerkin(int dim, int nx, int ny, const double *Af, double *Ac)
{
    galerkin_d(dim, nx, ny, Af, Ac);
}

/* V-cycles in FP64, or in FP32 when p->inner_fp32 (A0, b0 and x rounded to
 * float on entry, x returned in double). */
int orc_vcycles(int dim, int nx, int ny, const orc_params *p, const double *A0,
                const double *b0, double *x, int n_cycles)
{
    if (p->inner_fp32) return vcycles_f(dim, nx, ny, p, A0, b0, x, n_cycles);
    return vcycles_d(dim, nx, ny, p, A0, b0, x, n_cycles);
}

/* ------------------------------------------------------------------------ */
/* Dry-cell remark of Sec. 2.4: a cell with h < h_eps is reset to zero. */
static void threshold_cell(const prob *P, double *U, int idx)
{
    if (U[idx] < P->p->h_eps)
        for (int k = 0; k < P->nc; ++k) U[k * P->N + idx] = 0.0;
}

void orc_threshold(const orc_grid *gr, const orc_params *p, double *U)
{
    prob P;
    orc_side dummy[4];
    memset(dummy, 0, sizeof dummy);
    if (setup(&P, gr, dummy, p, NULL)) return;
    ORC_PARALLEL_FOR
    for (int idx = 0; idx < P.N; ++idx) threshold_cell(&P, U, idx);
}

/* BLU-SGS update of one cell (Algorithm 1, Step 2.1): with R_i and dR_i/dU_i
 * evaluated at the latest states, U_i -= (alpha ||R_i||_1 I + dR_i/dU_i)^{-1} R_i,
 * then the dry threshold. */
static void blu_cell(const prob *P, double *U, int i, int j)
{
    int idx = j * P->gr->nx + i, nc = P->nc;
    double Rc[3], Dm[3][3], M[9], d[3];
    cell_jacobian(P, U, i, j, Rc, Dm, NULL);
    double nrm = l1(nc, Rc);
    for (int r = 0; r < nc; ++r) Dm[r][r] = Dm[r][r] + P->p->alpha * nrm;
    if (P->p->dry_pin && U[idx] == 0.0) dry_momentum_pin(nc, Rc, Dm, NULL);
    for (int r = 0; r < nc; ++r)
        for (int c = 0; c < nc; ++c) M[r * nc + c] = Dm[r][c];
    orc_solve_block(nc, M, Rc, d);
    for (int k = 0; k < nc; ++k) U[k * P->N + idx] = U[k * P->N + idx] - d[k];
    threshold_cell(P, U, idx);
}

static void blu_half(const prob *P, double *U, int color)
{
    ORC_PARALLEL_FOR
    for (int j = 0; j < P->gr->ny; ++j)
        for (int i = 0; i < P->gr->nx; ++i)
            if (((i + j) & 1) == color) blu_cell(P, U, i, j);
}

/* One symmetric BLU-SGS sweep: lexicographic forward then backward, or
 * red, black, black, red. */
int orc_blu_sweep(const orc_grid *gr, const orc_side bc[4], const orc_params *p,
                  const double *z, double *U)
{
    prob P;
    if (setup(&P, gr, bc, p, z)) return ORC_EINVAL;
    if (p->order == ORC_LEX) {
        for (int idx = 0; idx < P.N; ++idx) blu_cell(&P, U, idx % gr->nx, idx / gr->nx);
        for (int idx = P.N - 1; idx >= 0; --idx) blu_cell(&P, U, idx % gr->nx, idx / gr->nx);
    } else {
        blu_half(&P, U, 0);
        blu_half(&P, U, 1);
        blu_half(&P, U, 1);
        blu_half(&P, U, 0);
    }
    return ORC_OK;
}

/* Relaxed update of eq:NewtonREG-12, U_i += tau_i dU_i, with the per-cell
 * relaxation tau_i = tau except where the step would take more than the
 * fraction pos_theta of the cell's depth away: there
 * tau_i = pos_theta * h_i / (-dh_i).  (pos_theta = 0 gives tau_i = tau.) */
static void relaxed_update(const prob *P, double *U, const double *x)
{
    double th = P->p->pos_theta, tau = P->p->tau;
    ORC_PARALLEL_FOR
    for (int idx = 0; idx < P->N; ++idx) {
        double t = tau;
        double h = U[idx], dh = x[idx];
        if (th > 0.0 && dh < 0.0 && h + tau * dh < (1.0 - th) * h) t = th * h / (-dh);
        for (int k = 0; k < P->nc; ++k) U[k * P->N + idx] = U[k * P->N + idx] + t * x[k * P->N + idx];
    }
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1, Step 1: the initial data averaged onto the coarsest mesh, then
 * on each level l = N_L, ..., 1 symmetric BLU-SGS iterations until
 * sum_i ||R_{i,l}||_1 < eps_p 2^-l, and the result injected into the children
 * on level l - 1.  Coarse meshes cover the same domain with (nx, ny) >> l;
 * their bed and initial state are averages of the children, taken level by
 * level in the child order SW, SE, NW, NE as (((SW + SE) + NW) + NE) / 4
 * (1D: (left + right) / 2).  The residual is tested before each sweep; at
 * most init_max_sweeps sweeps per level. */

static void average_children(int dim, int nxf, int nyf, int ncomp, const double *f, double *c)
{
    int nxc = nxf / 2, nyc = dim == 1 ? 1 : nyf / 2;
    int Nf = nxf * nyf, Nc = nxc * nyc;
    for (int k = 0; k < ncomp; ++k)
        for (int J = 0; J < nyc; ++J)
            for (int I = 0; I < nxc; ++I) {
                const double *q = f + (size_t)k * Nf;
                double v;
                if (dim == 1) {
                    v = (q[2 * I] + q[2 * I + 1]) * 0.5;
                } else {
                    int r0 = 2 * J * nxf, r1 = (2 * J + 1) * nxf;
                    v = (((q[r0 + 2 * I] + q[r0 + 2 * I + 1]) + q[r1 + 2 * I]) + q[r1 + 2 * I + 1]) * 0.25;
                }
                c[(size_t)k * Nc + J * nxc + I] = v;
            }
}

static void inject_children(int dim, int nxf, int nyf, int ncomp, const double *c, double *f)
{
    int nxc = nxf / 2, nyc = dim == 1 ? 1 : nyf / 2;
    int Nf = nxf * nyf, Nc = nxc * nyc;
    for (int k = 0; k < ncomp; ++k)
        for (int j = 0; j < nyf; ++j)
            for (int i = 0; i < nxf; ++i)
                f[(size_t)k * Nf + j * nxf + i] = c[(size_t)k * Nc + (dim == 1 ? 0 : j / 2) * nxc + i / 2];
}

int orc_nested_init(const orc_grid *gr, const orc_side bc[4], const orc_params *p,
                    const double *z, double *U, int *sweeps)
{
    const int NL = p->n_levels, nc = gr->dim == 1 ? 2 : 3;
    if (sweeps)
        for (int l = 0; l <= NL; ++l) sweeps[l] = 0;
    if (!(p->eps_p > 0.0) || NL < 1) return ORC_OK;
    orc_grid G[16];
    double *zl[16], *Ul[16];
    G[0] = *gr;
    zl[0] = (double *)z;
    Ul[0] = U;
    int rc = ORC_OK;
    for (int l = 1; l <= NL; ++l) {
        G[l] = G[l - 1];
        G[l].nx = G[l - 1].nx / 2;
        G[l].ny = gr->dim == 1 ? 1 : G[l - 1].ny / 2;
        size_t N = (size_t)G[l].nx * G[l].ny;
        zl[l] = (double *)malloc(sizeof(double) * N);
        Ul[l] = (double *)malloc(sizeof(double) * N * nc);
        if (!zl[l] || !Ul[l]) {
            for (int q = 1; q <= l; ++q) { free(zl[q]); free(Ul[q]); }
            return ORC_EINVAL;
        }
        average_children(gr->dim, G[l - 1].nx, G[l - 1].ny, 1, zl[l - 1], zl[l]);
        average_children(gr->dim, G[l - 1].nx, G[l - 1].ny, nc, Ul[l - 1], Ul[l]);
    }
    for (int l = NL; l >= 1 && rc == ORC_OK; --l) {
        const double thr = ldexp(p->eps_p, -l);
        int cnt = 0;
        for (;;) {
            double res = 0.0;
            rc = orc_residual(&G[l], bc, p, zl[l], Ul[l], NULL, &res);
            if (rc || !(res >= thr) || cnt >= p->init_max_sweeps) break;
            rc = orc_blu_sweep(&G[l], bc, p, zl[l], Ul[l]);
            if (rc) break;
            ++cnt;
        }
        if (sweeps) sweeps[l] = cnt;
        inject_children(gr->dim, G[l - 1].nx, G[l - 1].ny, nc, Ul[l], Ul[l - 1]);
    }
    for (int l = 1; l <= NL; ++l) { free(zl[l]); free(Ul[l]); }
    return rc;
}

/* Algorithm 1, Steps 2-3, started from the given U (Step 1 is not part of
 * this routine).  Each Newton step: optional BLU-SGS pre-smoothing, assembly
 * of R and A at the current U, stop test on sum_i ||R_i||_1, N_mg V-cycles
 * from dU = 0, relaxed update U += tau dU and the dry threshold. */
int orc_newton_solve(const orc_grid *gr, const orc_side bc[4], const orc_params *p,
                     const double *z, double *U, double tol, orc_stats *st)
{
    prob P;
    if (setup(&P, gr, bc, p, z)) return ORC_EINVAL;
    int dim = gr->dim, nx = gr->nx, ny = gr->ny, nc = P.nc, nb = P.nf + 1;
    size_t nv = (size_t)nc * P.N;
    double *A = (double *)malloc(sizeof(double) * nb * nc * nc * P.N);
    double *b = (double *)malloc(sizeof(double) * nv);
    double *Ulast = (double *)malloc(sizeof(double) * nv);
    unsigned char *iso = (unsigned char *)malloc((size_t)P.N);
    int status = ORC_NOT_CONVERGED, n = 0;
    double res = 0.0, res0 = 0.0;
    if (st) { st->newton_steps = 0; st->n_pinned = 0; st->res_l1 = 0.0; st->init_sweeps = 0; }
    orc_threshold(gr, p, U);
    if (p->eps_p > 0.0 && p->n_levels >= 1) {      /* Step 1 */
        int sw[16];
        if (orc_nested_init(gr, bc, p, z, U, sw)) { free(A); free(b); free(Ulast); free(iso); return ORC_EINVAL; }
        if (st)
            for (int l = 1; l <= p->n_levels; ++l) st->init_sweeps += sw[l];
    }
    for (n = 0; n < p->max_newton; ++n) {
        memcpy(Ulast, U, sizeof(double) * nv);
        for (int s = 0; s < p->blu_sweeps; ++s) orc_blu_sweep(gr, bc, p, z, U);
        orc_assemble(gr, bc, p, z, U, A, b, &res);
        if (st && st->res_hist && n < st->hist_cap) st->res_hist[n] = res;
        if (n == 0) res0 = res;
        if (!isfinite(res)) { memcpy(U, Ulast, sizeof(double) * nv); status = ORC_ENONFINITE; break; }
        if (res < tol) { status = ORC_OK; break; }
        if (res > 1e8 * res0) { status = ORC_EDIVERGED; break; }
        double *x = (double *)calloc(nv, sizeof(double));
        if (orc_vcycles(dim, nx, ny, p, A, b, x, p->n_mg)) { free(x); status = ORC_EINVAL; break; }
        relaxed_update(&P, U, x);
        free(x);
        orc_threshold(gr, p, U);
    }
    if (status == ORC_NOT_CONVERGED) orc_residual(gr, bc, p, z, U, NULL, &res);
    if (st) {
        orc_isolated(gr, bc, p, z, U, iso);
        int cnt = 0;
        for (int q = 0; q < P.N; ++q) cnt += iso[q];
        st->n_pinned = cnt;
        st->newton_steps = n;
        st->status = status;
        st->res_l1 = res;
    }
    free(A); free(b); free(Ulast); free(iso);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Sensitivities.  At a steady state R(U, z) = 0 (eq:Res), an objective
 * J(U, z) has the bed derivative dJ/dz = dJ/dz|_U - lam^T dR/dz, where lam
 * solves (dR/dU)^T lam = (dJ/dU)^T and dR/dU is the assembled Newton matrix
 * of eq:MatrixForm (the linearization the solver itself uses).  Pinned rows
 * of that matrix (isolated cells, the momentum of exactly dry cells) are
 * unknowns held fixed by the linearization, so their rows of dR/dz are
 * pinned the same way. */

static const int OPP[4] = {FE, FW, FN, FS};   /* face of the neighbour that faces back */

void orc_transpose_blocks(int dim, int nx, int ny, const double *A, double *At)
{
    int nc = dim == 1 ? 2 : 3, nf = dim == 1 ? 2 : 4, N = nx * ny, ni, nj;
#define TIDX(b, r, c, idx) ((((size_t)(b) * nc + (r)) * nc + (c)) * N + (idx))
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            int idx = j * nx + i;
            for (int r = 0; r < nc; ++r)
                for (int c = 0; c < nc; ++c) {
                    At[TIDX(0, r, c, idx)] = A[TIDX(0, c, r, idx)];
                    for (int f = 0; f < nf; ++f) {
                        double v = 0.0;
                        if (nbr(dim, nx, ny, i, j, f, &ni, &nj))
                            v = A[TIDX(OPP[f] + 1, c, r, nj * nx + ni)];
                        At[TIDX(f + 1, r, c, idx)] = v;
                    }
                }
        }
#undef TIDX
}

/* Row pins of the Newton matrix applied to one row's bed derivative d. */
static void pin_row(const prob *P, const unsigned char *iso, const double *U, int idx, double *d)
{
    if (iso[idx]) {
        for (int r = 0; r < P->nc; ++r) d[r] = 0.0;
    } else if (P->p->dry_pin && U[idx] == 0.0) {
        for (int r = 1; r < P->nc; ++r) d[r] = 0.0;
    }
}

/* For each cell j, with its bed raised to z_j + eps (eps = fd_eps, the
 * absolute step of eq:NumerDiff):
 *   dR_j/dz_j = sum over j's faces (W, E, S, N) of |e| (T(z_j + eps) - T) / eps,
 *     a boundary face's ghost carrying the raised bed (ghost bed = own bed);
 *   dR_i/dz_j = |e| (T(z_j + eps) - T) / eps for each neighbour i, T being i's
 *     edge term on its face towards j;
 * then out_j = lam_j . dR_j/dz_j + sum over j's neighbours (W, E, S, N) of
 * lam_i . dR_i/dz_j, each dot product over the components in order. */
int orc_bed_vjp(const orc_grid *gr, const orc_side bc[4], const orc_params *p,
                const double *z, const double *U, const double *lam, double *out)
{
    prob P;
    if (setup(&P, gr, bc, p, z)) return ORC_EINVAL;
    int nx = gr->nx, ny = gr->ny, nc = P.nc, N = P.N, ni, nj;
    double *zw = (double *)malloc(sizeof(double) * (size_t)N);
    unsigned char *iso = (unsigned char *)malloc((size_t)N);
    if (!zw || !iso) { free(zw); free(iso); return ORC_EINVAL; }
    memcpy(zw, z, sizeof(double) * (size_t)N);
    orc_isolated(gr, bc, p, z, U, iso);
    P.z = zw;
    const double eps = p->fd_eps;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            int idx = j * nx + i;
            double Uo[3], Un[3] = {0, 0, 0}, T0[3], Tp[3], d[3];
            load_cell(&P, U, idx, Uo);
            for (int r = 0; r < nc; ++r) d[r] = 0.0;
            for (int f = 0; f < P.nf; ++f) {
                double e = P.elen[f];
                if (nbr(gr->dim, nx, ny, i, j, f, &ni, &nj)) load_cell(&P, U, nj * nx + ni, Un);
                cell_edge(&P, i, j, f, Uo, Un, T0);
                zw[idx] = z[idx] + eps;
                cell_edge(&P, i, j, f, Uo, Un, Tp);
                zw[idx] = z[idx];
                for (int r = 0; r < nc; ++r) d[r] = d[r] + e * ((Tp[r] - T0[r]) / eps);
            }
            pin_row(&P, iso, U, idx, d);
            double acc = 0.0;
            for (int r = 0; r < nc; ++r) acc = acc + lam[r * N + idx] * d[r];
            for (int f = 0; f < P.nf; ++f) {
                if (!nbr(gr->dim, nx, ny, i, j, f, &ni, &nj)) continue;
                int nidx = nj * nx + ni, g = OPP[f];
                double e = P.elen[g];
                load_cell(&P, U, nidx, Un);
                cell_edge(&P, ni, nj, g, Un, Uo, T0);
                zw[idx] = z[idx] + eps;
                cell_edge(&P, ni, nj, g, Un, Uo, Tp);
                zw[idx] = z[idx];
                for (int r = 0; r < nc; ++r) d[r] = e * ((Tp[r] - T0[r]) / eps);
                pin_row(&P, iso, U, nidx, d);
                for (int r = 0; r < nc; ++r) acc = acc + lam[r * N + nidx] * d[r];
            }
            out[idx] = acc;
        }
    free(zw);
    free(iso);
    return ORC_OK;
}
