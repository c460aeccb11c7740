// Host driver of the MI355X Newton multigrid library: the C ABI of
// include/nmg.h, the multigrid hierarchy, Algorithm 0 (V-cycle) and
// Algorithm 1 Steps 2-3 (Newton loop) of Wu & Tang (arXiv:1608.06721).
#include "nmg.h"
#include "nmg_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

using namespace nmg;

static_assert(sizeof(((nmg_stats *)nullptr)->init_level_sweeps) == kMaxLevels * sizeof(int),
              "one Step 1 sweep count per level");

namespace {

// State of one colour of a level's correction vector x.
enum ColorState {
    ST_VALID = 0,       // stored values are the current ones
    ST_ZERO = 1,        // current value is 0 (not materialized)
    ST_VALID_PP = 2,    // stored values + pending prolongation of the coarse correction
    ST_ZERO_PP = 3      // 0 + pending prolongation
};

struct Level {
    LevelGeom G;
    void *A = nullptr, *b = nullptr, *x = nullptr;   // double, or float (FP32 inner)
    void *xt = nullptr;     // one colour's planes: the other buffer of fused half-sweep pairs
    int st[2] = {ST_ZERO, ST_ZERO};
    int last = -1;      // colour of the last half sweep if nothing changed since, else -1
};

}  // namespace

struct nmg_batch;

struct nmg_ctx {
    nmg_grid grid;
    nmg_bc bc;
    nmg_params prm;
    hipStream_t stream = nullptr;
    Phys P;
    int dim = 0, nc = 0, nb = 0, ne = 0, NL = 0;
    bool f32 = false;                 // FP32 inner V-cycle
    int fuse = 3;                     // most half sweeps per launch on launched coarse levels
    int split = 1;                    // coarsest-level runs may use two lanes per cell
    int blu_lanes = -1;               // lanes per cell of BLU-SGS half sweeps (-1: by mesh)
    int step1_graph = 1;              // Step 1 runs of kStep1Ahead sweeps replayed as graphs
    Level L[16];
    void *pool = nullptr;             // the hierarchy's allocation
    // Residuals of colour res_color of level res_level (res_level -1: none
    // valid), written by the last half sweep of a pre-smoothing for the
    // restriction that follows it: NC planes of level 0's size in the
    // hierarchy's type (a batch's template instance points at the batch's
    // per-instance planes instead, through its level table).
    void *rres = nullptr;
    int res_level = -1, res_color = -1;
    void *At_alloc = nullptr;         // second level-0 matrix (adjoint transpose), owned
    void *At_spare = nullptr;         // whichever of the two level-0 matrices is not L[0].A
    // Algorithm 1, Step 1 (allocated on first use): coarse beds and states
    double *init_pool = nullptr;
    double *zl[kMaxLevels] = {}, *Ul[kMaxLevels] = {};
    double *init_red = nullptr;     // Step 1: first half sweep's red states
    double *init_part = nullptr;    // Step 1: residual partials of that launch
    hipStream_t cap_stream = nullptr;                 // Step 1 graph capture
    hipGraphExec_t init_graph[kMaxLevels] = {};       // Step 1 run of sweeps, per level
    // Krylov acceleration of the adjoint solve (allocated on first use)
    int km = 0;                       // restart length the buffers were sized for
    double *kV = nullptr, *kg = nullptr, *kx = nullptr, *kw = nullptr;
    double *kpart = nullptr, *kdots = nullptr, *kcoef = nullptr, *h_k = nullptr;
    unsigned char *iso = nullptr;
    double *partial = nullptr;    // per-block partial sums
    double *scal = nullptr;       // device scalars
    double *h_scal = nullptr;     // pinned host mirror
    double *Ulast = nullptr;      // U before the current Newton step
    std::string err;
    // measurement hooks
    bool timing = false;
    int nrec = 0;                 // event pairs of ev[] in use
    int tgroup = -1;              // pair of the open run of back-to-back timed launches, or -1
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    std::vector<long long> ev_cells;
    std::vector<int> ev_launches;
    // phase boundaries of the Newton solve: event k closes phase pev_ph[k]
    // (NMG_PHASE_*, or -1 for the start of a solve), which began at event k-1
    std::vector<hipEvent_t> pev;
    std::vector<signed char> pev_ph;
    int npev = 0;
    // coarse part of the V-cycle in one workgroup (levels lc..NL), recorded
    // once from the same state machine that drives the per-level launches
    int lc = -1;
    bool recording = false;
    std::vector<CoarseOp> rec;
    int prog_len = 0;                 // operations of the recorded coarse program (rec)
    int l_lds = -1;                   // levels l_lds..NL run from LDS in the coarse kernel
    CoarseOp *d_ops = nullptr;
    LevelDev *d_lv = nullptr;
    // set on the first instance of a batch: its state machine then drives
    // batched launches over every instance
    nmg_batch *batch = nullptr;
};

struct nmg_batch {
    int n = 0, dim = 0, nc = 0, NL = 0;
    bool f32 = false;
    hipStream_t stream = nullptr;
    nmg_params prm;
    std::string err;
    std::vector<nmg_ctx *> inst;          // inst[0]'s state machine drives the batch
    std::vector<BatchInst> h_inst;
    BatchInst *d_inst = nullptr;
    BatchLevel *d_lv = nullptr;           // [(NL + 1) * n], level-major
    void *d_rr = nullptr;                 // each instance's residual planes (level 0's size)
    LevelDev *d_clv = nullptr;            // [n * kMaxLevels] coarse-kernel level tables
    WorkItem *d_work = nullptr;
    WorkRange w_cells0{nullptr, 0};       // 256-cell tiles of level 0
    WorkRange w_plane[kMaxLevels][kNumTiles];   // colour-plane tiles per tile length
    WorkRange w_ccells[kMaxLevels];       // 256-cell tiles of level l (Galerkin into l)
    WorkRange w_rchild[kMaxLevels];       // tiles of 256 children of level l's cells (restriction into l)
    WorkRange w_tile2d[kMaxLevels];       // 32x16 cell tiles of level l (fused half-sweep pairs)
    long cells_l[kMaxLevels] = {};        // cells of level l summed over the instances
    int tile[kMaxLevels];                 // tile length of the half sweeps per level
    int persist = 0;                      // blocks of the persistent half sweep (0: one per item)
    int *d_active = nullptr, *h_active = nullptr;   // instances still iterating
    int *d_mask = nullptr, *h_mask = nullptr;       // a second instance mask
    int *d_roff = nullptr, *d_rcnt = nullptr;       // each instance's level-0 tiles
    double *d_partial = nullptr, *d_norm = nullptr, *h_norm = nullptr;
};

namespace {

int fail(nmg_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

// Measurement hook: an event on the stream that closes phase `ph` of the
// Newton solve (-1: the start of a solve, attributed to no phase).  Marks
// beyond the event pool are dropped.
int phase_mark(nmg_ctx *c, int ph)
{
    if (!c->timing || c->npev >= (int)c->pev.size()) return NMG_OK;
    if (hipEventRecord(c->pev[c->npev], c->stream) != hipSuccess)
        return fail(c, NMG_EHIP, "hipEventRecord failed");
    c->pev_ph[c->npev++] = (signed char)ph;
    return NMG_OK;
}

#define HIPCHK(ctx, call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, NMG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));  \
    } while (0)

long cells(const LevelGeom &G) { return (long)G.nx * G.ny; }

int check_params(const nmg_grid *g, const nmg_bc *bc, const nmg_params *p, std::string &msg)
{
    if (!g || !bc || !p) { msg = "null grid/bc/params"; return NMG_EINVAL; }
    if (g->dim != 1 && g->dim != 2) { msg = "dim must be 1 or 2"; return NMG_EINVAL; }
    if (g->nx < 2 || g->ny < 1 || (g->dim == 1 && g->ny != 1) || (g->dim == 2 && g->ny < 2)) {
        msg = "bad grid size";
        return NMG_EINVAL;
    }
    if (!(g->x1 > g->x0) || (g->dim == 2 && !(g->y1 > g->y0))) { msg = "empty domain"; return NMG_EINVAL; }
    if (p->n_levels < 0 || p->n_levels > 15) { msg = "n_levels out of range"; return NMG_EINVAL; }
    long div = 1L << p->n_levels;
    if (g->nx % div || (g->dim == 2 && g->ny % div)) {
        msg = "nx (and ny) must be divisible by 2^n_levels";
        return NMG_EINVAL;
    }
    if (p->flux != NMG_FLUX_HLL && p->flux != NMG_FLUX_LLF && p->flux != NMG_FLUX_HLLC) {
        msg = "unknown flux";
        return NMG_EINVAL;
    }
    if (!(p->g > 0) || !(p->fd_eps > 0) || !(p->alpha >= 0) || !(p->h_eps >= 0) || !(p->tau > 0) ||
        !(p->eps_r >= 0) || !(p->pos_theta >= 0 && p->pos_theta < 1)) {
        msg = "bad scalar parameter";
        return NMG_EINVAL;
    }
    if (p->inner_fp32 != 0 && p->inner_fp32 != 1) { msg = "inner_fp32 must be 0 or 1"; return NMG_EINVAL; }
    if (p->gamma < 1 || p->gamma > 3) { msg = "gamma must be 1, 2 or 3"; return NMG_EINVAL; }
    if (!(p->eps_p >= 0) || p->init_max_sweeps < 0) { msg = "bad eps_p or init_max_sweeps"; return NMG_EINVAL; }
    if (p->flux == NMG_FLUX_HLLC && g->dim != 2) { msg = "HLLC is a 2D flux"; return NMG_EINVAL; }
    if (p->nu1 < 0 || p->nu2 < 0 || p->nu_coarse < 0 || p->n_mg < 0 || p->blu_sweeps < 0 ||
        p->max_newton < 0) {
        msg = "negative iteration count";
        return NMG_EINVAL;
    }
    int nsides = g->dim == 1 ? 2 : 4;
    for (int f = 0; f < nsides; ++f) {
        const nmg_side &s = bc->side[f];
        if (s.kind < 0 || s.kind > 2) { msg = "bad boundary kind"; return NMG_EINVAL; }
        if (s.kind == NMG_BC_OPEN) {
            bool hq = !std::isnan(s.qn), hh = !std::isnan(s.h);
            if (!hq && !hh) { msg = "open side needs qn or h"; return NMG_EINVAL; }
            if (hq && !(s.qn > 0)) { msg = "inflow discharge qn must be > 0"; return NMG_EINVAL; }
            if (hh && !(s.h > 0)) { msg = "prescribed depth h must be > 0"; return NMG_EINVAL; }
        }
    }
    return NMG_OK;
}

// ---- multigrid on the colour-split hierarchy -----------------------------

// res: a restriction from level l follows this half sweep; a normal-mode
// launch then also writes the updated cells' residuals (c->rres), which the
// restriction reads instead of recomputing them.  Any other change to the
// level's x invalidates them.
int halfsweep(nmg_ctx *c, int l, int color, bool res = false)
{
    Level &Lv = c->L[l];
    if (Lv.last == color) return NMG_OK;   // same colour again: result identical, elide
    if (c->res_level == l) c->res_level = -1;
    int oc = color ^ 1;
    int mode;
    switch (Lv.st[oc]) {
    case ST_VALID: mode = MODE_NORMAL; break;
    case ST_ZERO: mode = MODE_ZERO; break;
    case ST_VALID_PP: mode = MODE_PROLONG; break;
    default: mode = MODE_PROLONG_ZERO; break;
    }
    const Level &Lc = c->L[l + 1 <= c->NL ? l + 1 : l];
    if (c->recording) {
        c->rec.push_back(CoarseOp{COP_SGS, l, color, mode});
        Lv.st[color] = ST_VALID;
        Lv.last = color;
        return NMG_OK;
    }
    res = res && mode == MODE_NORMAL && c->rres;
    if (c->batch) {
        nmg_batch *B = c->batch;
        const int tl = B->tile[l];
        int ti = 0;
        while (kTileChoices[ti] != tl) ++ti;
        if (res) {
            HIPCHK(c, launch_b_sgs_half_res(c->dim, c->f32, tl, B->d_lv + (long)l * B->n,
                                            B->w_plane[l][ti], B->d_active, color, c->stream));
            c->res_level = l;
            c->res_color = color;
        } else {
            HIPCHK(c, launch_b_sgs_half(c->dim, c->f32, mode, tl, B->d_lv + (long)l * B->n,
                                        B->w_plane[l][ti], B->d_active, color, B->persist,
                                        c->stream));
        }
        Lv.st[color] = ST_VALID;
        Lv.last = color;
        return NMG_OK;
    }
    // Measurement hook: full half sweeps (all neighbour blocks read) of the
    // finest level.  A run of them launched back to back (within one
    // smoothing call) shares one pair of events around the whole run.
    const bool want = c->timing && l == 0 && mode == MODE_NORMAL && !res;
    const bool open = want && c->tgroup >= 0;
    const int k = open ? c->tgroup : c->nrec;
    const bool rec = want && k < (int)c->ev.size();
    if (rec && !open) HIPCHK(c, hipEventRecord(c->ev[k].first, c->stream));
    if (res) {
        HIPCHK(c, launch_sgs_half_res(c->dim, c->f32, Lv.G, Lv.A, Lv.b, Lv.x, color, c->rres,
                                      stream_level(cells(Lv.G), c->nc, c->f32 ? 4 : 8),
                                      c->stream));
        c->res_level = l;
        c->res_color = color;
    } else {
        HIPCHK(c, launch_sgs_half(c->dim, c->f32, mode, Lv.G, Lv.A, Lv.b, Lv.x, color, Lc.G,
                                  Lc.x, stream_level(cells(Lv.G), c->nc, c->f32 ? 4 : 8),
                                  c->stream));
    }
    if (rec) {
        HIPCHK(c, hipEventRecord(c->ev[k].second, c->stream));
        long n = 0;
        for (int j = 0; j < Lv.G.ny; ++j) n += (Lv.G.nx - ((j + color) & 1) + 1) / 2;
        c->ev_cells[k] += n;
        c->ev_launches[k] += 1;
        if (!open) {
            c->nrec = k + 1;
            c->tgroup = k;
        }
    } else {
        c->tgroup = -1;
    }
    Lv.st[color] = ST_VALID;
    Lv.last = color;
    return NMG_OK;
}

int smooth_single(nmg_ctx *c, int l, int iters, bool res_last = false);

// Whether the half sweeps of level l are launched as fused pairs: 2D levels
// launched level by level whose half sweep is bound by launch latency rather
// than bandwidth (measured: a pair takes 6.7-8.0 us against 2 x 4.6-4.8 us
// up to 256x256, 21.5 us against 2 x 10.3 us at 512x512).
constexpr long kPairMaxCells = 1L << 17;
// Triples replace a pair and a single launch only on the smallest launched
// levels (measured: 9.4 us against 6.5 + 4.5 us at 64x64, 11.8 against
// 7.0 + 4.7 us at 128x128, 13.5 against 8.0 + 4.8 us at 256x256).
constexpr long kTripleMaxCells = 1L << 12;
long batch_cells(const nmg_ctx *c, int l) { return c->batch->cells_l[l]; }

bool fuse_pairs(const nmg_ctx *c, int l)
{
    if (c->recording || c->dim != 2 || l == 0) return false;
    if (c->lc >= 0 && l >= c->lc) return false;
    const long n = c->batch ? batch_cells(c, l) : cells(c->L[l].G);
    if (n > kPairMaxCells) return false;
    return c->fuse >= 2;
}

int sweep_mode(int st_other)
{
    switch (st_other) {
    case ST_VALID: return MODE_NORMAL;
    case ST_ZERO: return MODE_ZERO;
    case ST_VALID_PP: return MODE_PROLONG;
    default: return MODE_PROLONG_ZERO;
    }
}

// The half sweeps of `iters` symmetric iterations on level l (colour order
// 0, 1, 1, 0, a repeat of the last colour elided), fused into launches of two
// or three consecutive half sweeps.  Fused launches come in groups of two
// (pair + pair or pair + triple) that start on the same colour: the first
// reads the second colour from x and writes it to the level's xt, the second
// reads it from xt and writes it back to x, so the values end in x.  The
// rest are launched one by one; the plan uses the fewest launches.
int smooth_pairs(nmg_ctx *c, int l, int iters)
{
    Level &Lv = c->L[l];
    const Level &Lc = c->L[l + 1 <= c->NL ? l + 1 : l];
    constexpr int kMax = 64;
    int col[kMax], mode[kMax], k = 0;
    int st[2] = {Lv.st[0], Lv.st[1]}, last = Lv.last;
    const int order[4] = {0, 1, 1, 0};
    for (int it = 0; it < iters; ++it)
        for (int q = 0; q < 4; ++q) {
            const int cl = order[q];
            if (cl == last) continue;
            if (k == kMax) return smooth_single(c, l, iters);
            col[k] = cl;
            mode[k] = sweep_mode(st[cl ^ 1]);
            st[cl] = ST_VALID;
            last = cl;
            ++k;
        }
    // best[q]: fewest launches for half sweeps q..k-1; step[q]: 1 (single),
    // 4 (pair + pair) or 5 (pair + triple)
    int best[kMax + 1], step[kMax + 1];
    const bool triples = !c->batch && c->fuse >= 3 && cells(Lv.G) <= kTripleMaxCells;
    best[k] = 0;
    for (int q = k - 1; q >= 0; --q) {
        best[q] = 1 + best[q + 1];
        step[q] = 1;
        if (q + 4 <= k && 2 + best[q + 4] < best[q]) { best[q] = 2 + best[q + 4]; step[q] = 4; }
        if (triples && q + 5 <= k && 2 + best[q + 5] < best[q]) {
            best[q] = 2 + best[q + 5];
            step[q] = 5;
        }
    }
    const size_t esz = c->f32 ? sizeof(float) : sizeof(double);
    for (int q = 0; q < k;) {
        if (step[q] == 1) {
            int rc = halfsweep(c, l, col[q]);
            if (rc) return rc;
            ++q;
            continue;
        }
        const int c1 = col[q], c2 = c1 ^ 1;
        if (c->batch) {
            const nmg_batch *B = c->batch;
            const BatchLevel *blv = B->d_lv + (long)l * B->n;
            HIPCHK(c, launch_b_sgs_pair(c->f32, mode[q], blv, B->w_tile2d[l], B->d_active, c1, 0,
                                        c->stream));
            HIPCHK(c, launch_b_sgs_pair(c->f32, MODE_NORMAL, blv, B->w_tile2d[l], B->d_active, c1,
                                        1, c->stream));
            Lv.st[0] = Lv.st[1] = ST_VALID;
            Lv.last = c2;
            q += 4;
            continue;
        }
        void *xc2 = (char *)Lv.x + (size_t)c2 * c->nc * Lv.G.plane * esz;
        HIPCHK(c, launch_sgs_pair(c->f32, mode[q], Lv.G, Lv.A, Lv.b, Lv.x, xc2, Lv.xt, c1,
                                  Lc.G, Lc.x, c->stream));
        if (step[q] == 4)
            HIPCHK(c, launch_sgs_pair(c->f32, MODE_NORMAL, Lv.G, Lv.A, Lv.b, Lv.x, Lv.xt, xc2,
                                      c1, Lc.G, Lc.x, c->stream));
        else
            HIPCHK(c, launch_sgs_triple(c->f32, MODE_NORMAL, Lv.G, Lv.A, Lv.b, Lv.x, Lv.xt, xc2,
                                        c1, Lc.G, Lc.x, c->stream));
        Lv.st[0] = Lv.st[1] = ST_VALID;
        Lv.last = step[q] == 4 ? c2 : c1;
        q += step[q];
    }
    return NMG_OK;
}

// res_last: a restriction from level l follows (see halfsweep).
int smooth(nmg_ctx *c, int l, int iters, bool res_last = false)
{
    if (fuse_pairs(c, l)) return smooth_pairs(c, l, iters);
    return smooth_single(c, l, iters, res_last);
}

int smooth_single(nmg_ctx *c, int l, int iters, bool res_last)
{
    c->tgroup = -1;               // timed runs never span other launches
    for (int it = 0; it < iters; ++it) {
        int rc;
        if ((rc = halfsweep(c, l, 0)) || (rc = halfsweep(c, l, 1)) || (rc = halfsweep(c, l, 1)) ||
            (rc = halfsweep(c, l, 0, res_last && it + 1 == iters)))
            return rc;
    }
    c->tgroup = -1;
    return NMG_OK;
}

// Bring both colours of level l's x to stored, current values.
int materialize(nmg_ctx *c, int l)
{
    Level &Lv = c->L[l];
    const Level &Lc = c->L[l + 1 <= c->NL ? l + 1 : l];
    for (int color = 0; color < 2; ++color) {
        int op = -1;
        if (Lv.st[color] == ST_ZERO) op = 0;
        else if (Lv.st[color] == ST_VALID_PP) op = 1;
        else if (Lv.st[color] == ST_ZERO_PP) op = 2;
        if (op < 0) continue;
        if (c->res_level == l) c->res_level = -1;
        if (c->recording) {
            c->rec.push_back(CoarseOp{COP_FIX, l, color, op});
        } else if (c->batch) {
            nmg_batch *B = c->batch;
            int ti = 0;
            while (kTileChoices[ti] != kBlock) ++ti;
            HIPCHK(c, launch_b_fix_color(c->dim, c->f32, op, B->d_lv + (long)l * B->n,
                                         B->w_plane[l][ti], B->d_active, color, c->stream));
        } else {
            HIPCHK(c, launch_fix_color(c->dim, c->f32, op, Lv.G, Lv.x, color, Lc.G, Lc.x, c->stream));
        }
        Lv.st[color] = ST_VALID;
        Lv.last = -1;
    }
    return NMG_OK;
}

void set_zero(nmg_ctx *c, int l)
{
    c->L[l].st[0] = c->L[l].st[1] = ST_ZERO;
    c->L[l].last = -1;
    if (c->res_level == l) c->res_level = -1;
}

// Algorithm 0 with gamma = 1 (V-cycle) on level l.
int cycle(nmg_ctx *c, int l)
{
    const nmg_params &p = c->prm;
    int rc;
    c->res_level = -1;
    if ((rc = smooth(c, l, p.nu1, l < c->NL && !c->recording))) return rc;
    if (l == c->NL) {
        if ((rc = smooth(c, l, p.nu_coarse))) return rc;
    } else {
        if ((rc = materialize(c, l))) return rc;
        Level &Lv = c->L[l];
        Level &Lc = c->L[l + 1];
        if (c->recording)
            c->rec.push_back(CoarseOp{COP_RESTRICT, l, 0, 0});
        else if (c->batch && c->res_level == l)
            HIPCHK(c, launch_b_restrict_res(c->dim, c->f32,
                                            c->batch->d_lv + (long)l * c->batch->n,
                                            c->batch->w_rchild[l + 1], c->batch->d_active,
                                            c->res_color, c->stream));
        else if (c->batch)
            HIPCHK(c, launch_b_restrict(c->dim, c->f32, c->batch->d_lv + (long)l * c->batch->n,
                                        c->batch->w_rchild[l + 1], c->batch->d_active, c->stream));
        else if (c->res_level == l)
            HIPCHK(c, launch_restrict_res(c->dim, c->f32, Lv.G, Lv.A, Lv.b, Lv.x, Lc.G, Lc.b,
                                          c->rres, c->res_color,
                                          stream_level(cells(Lv.G), c->nc, c->f32 ? 4 : 8),
                                          c->stream));
        else
            HIPCHK(c, launch_restrict(c->dim, c->f32, Lv.G, Lv.A, Lv.b, Lv.x, Lc.G, Lc.b,
                                      stream_level(cells(Lv.G), c->nc, c->f32 ? 4 : 8),
                                      c->stream));
        c->res_level = -1;
        set_zero(c, l + 1);
        if (l + 1 == c->lc && !c->recording && c->prog_len > 0) {
            // The coarse calls below, from level lc down, run in one
            // workgroup (the program recorded by record_coarse) and leave
            // level lc's correction materialized.
            if (c->batch)
                HIPCHK(c, launch_b_coarse_cycle(c->dim, c->f32, c->d_ops, c->prog_len,
                                                c->batch->d_clv, c->batch->n,
                                                c->batch->d_active, c->l_lds, c->NL, c->stream));
            else
                HIPCHK(c, launch_coarse_cycle(c->dim, c->f32, c->d_ops, c->prog_len, c->d_lv,
                                              c->l_lds, c->NL,
                                              c->stream));
            Lc.st[0] = Lc.st[1] = ST_VALID;
            Lc.last = -1;
        } else {
            // gamma coarse cycles (gamma = 1: V, 2: W), one when leaving the
            // finest level (Algorithm 0)
            const int calls = (l == 0) ? 1 : p.gamma;
            for (int g = 0; g < calls; ++g)
                if ((rc = cycle(c, l + 1))) return rc;
            if ((rc = materialize(c, l + 1))) return rc;
        }
        for (int color = 0; color < 2; ++color)
            Lv.st[color] = (Lv.st[color] == ST_ZERO) ? ST_ZERO_PP : ST_VALID_PP;
        Lv.last = -1;
    }
    return smooth(c, l, p.nu2);
}

int build_coarse(nmg_ctx *c)
{
    for (int l = 1; l <= c->NL; ++l) {
        if (c->batch)
            HIPCHK(c, launch_b_galerkin(c->dim, c->f32, c->batch->d_lv + (long)(l - 1) * c->batch->n,
                                        c->batch->w_ccells[l], c->batch->d_active, c->stream));
        else
            HIPCHK(c, launch_galerkin(c->dim, c->f32, c->L[l - 1].G, c->L[l - 1].A, c->L[l].G,
                                      c->L[l].A, c->stream));
    }
    for (int l = 0; l <= c->NL; ++l) set_zero(c, l);
    return NMG_OK;
}

// Record the operations of the sub-cycle from level lc (which always starts
// from a zero correction) and upload them with the level table.
// Replace each maximal sequence of alternating half sweeps on the coarsest
// level (normal, or zero start first) by one COP_RUN, when that level is in
// LDS and has a thread per cell in the coarse-cycle kernel.
void merge_runs(nmg_ctx *c, bool fits)
{
    const int nl = c->NL;
    if (c->l_lds < 0 || !fits) return;
    std::vector<CoarseOp> out;
    const CoarseOp *r = c->rec.data();
    const int n = (int)c->rec.size();
    for (int q = 0; q < n;) {
        CoarseOp o = r[q];
        if (o.kind == COP_SGS && o.level == nl && (o.mode == MODE_NORMAL || o.mode == MODE_ZERO)) {
            int e = q + 1;
            while (e < n && r[e].kind == COP_SGS && r[e].level == nl && r[e].mode == MODE_NORMAL &&
                   r[e].color == (r[e - 1].color ^ 1))
                ++e;
            o.kind = COP_RUN;
            o.count = e - q;
            o.aux = c->split;
            q = e;
        } else {
            ++q;
        }
        out.push_back(o);
    }
    c->rec.swap(out);
    c->prog_len = (int)c->rec.size();
}

// Replace each maximal sequence of alternating half sweeps on the first
// coarse level lc (the first in any mode, the rest normal), with the
// restriction from lc when it follows, by one COP_REGRUN whose x and
// residual exchange area starts at LDS byte rs_off.  ok: lc lives in global memory,
// has at most one slot per colour and thread, and the exchange area fits.
void merge_reg_runs(nmg_ctx *c, bool ok, long rs_off)
{
    if (!ok) return;
    if (const char *e = std::getenv("NMG_COARSE_REG"))
        if (std::atoi(e) == 0) return;
    const int lc = c->lc;
    std::vector<CoarseOp> out;
    const CoarseOp *r = c->rec.data();
    const int n = (int)c->rec.size();
    for (int q = 0; q < n;) {
        CoarseOp o = r[q];
        if (o.kind == COP_SGS && o.level == lc) {
            int e = q + 1;
            while (e < n && r[e].kind == COP_SGS && r[e].level == lc && r[e].mode == MODE_NORMAL &&
                   r[e].color == (r[e - 1].color ^ 1))
                ++e;
            o.kind = COP_REGRUN;
            o.count = e - q;
            o.aux = 0;
            o.lds_off = (int)rs_off;
            if (e < n && r[e].kind == COP_RESTRICT && r[e].level == lc) {
                o.aux = 1;
                ++e;
            }
            q = e;
        } else {
            ++q;
        }
        out.push_back(o);
    }
    c->rec.swap(out);
    c->prog_len = (int)c->rec.size();
}

// LDS bytes of the coarse-cycle kernel's level copies (levels l_lds..NL).
long lds_levels_bytes(const nmg_ctx *c, int l_lds)
{
    long tot = 0;
    if (l_lds >= 0)
        for (int l = l_lds; l <= c->NL; ++l)
            tot += lds_level_bytes(c->L[l].G, c->ne, c->nc, c->f32 ? 4 : 8);
    return tot;
}

// Bytes of the LDS area (x, then the residual exchange) of a register-resident
// run on level l.
long reg_exchange_bytes(const nmg_ctx *c, int l)
{
    return 2L * c->nc * c->L[l].G.plane * (c->f32 ? 4 : 8);
}

// Whether level lc of context c can run as COP_REGRUN with its exchange area
// at LDS byte rs_off.
bool reg_run_fits(const nmg_ctx *c, int lc, int l_lds, long rs_off)
{
    if (l_lds >= 0 && lc >= l_lds) return false;
    if (c->L[lc].G.plane > kCoarseBlock) return false;
    return rs_off + reg_exchange_bytes(c, lc) <= kCoarseLdsBytes;
}

long coarse_cells_limit()
{
    long maxcells = 1024;
    if (const char *e = std::getenv("NMG_COARSE_CELLS")) maxcells = std::atol(e);
    return maxcells;
}

// First level at or below which the cycle runs in the coarse-cycle kernel.
int first_coarse_level(const nmg_ctx *c)
{
    const long maxcells = coarse_cells_limit();
    for (int l = 1; l <= c->NL; ++l)
        if (cells(c->L[l].G) <= maxcells) return l;
    return -1;
}

// Coarsest-first levels whose LDS copies fit the kernel (l_lds..NL), or -1.
int lds_first_level(const nmg_ctx *c, int lc)
{
    const long esz = c->f32 ? 4 : 8;
    long tot = 0;
    int l_lds = -1;
    for (int l = c->NL; l >= lc; --l) {
        tot += lds_level_bytes(c->L[l].G, c->ne, c->nc, esz);
        if (tot > kCoarseLdsBytes) break;
        l_lds = l;
    }
    return l_lds;
}

// The coarse-kernel level table of context c with levels l_lds..NL in LDS.
void coarse_level_table(const nmg_ctx *c, int l_lds, LevelDev *lv)
{
    long off = 0;
    for (int l = 0; l < kMaxLevels; ++l) {
        const Level &Lv = c->L[l <= c->NL ? l : c->NL];
        lv[l] = LevelDev{Lv.G, Lv.A, Lv.b, Lv.x, -1};
        if (l_lds >= 0 && l >= l_lds && l <= c->NL) {
            lv[l].lds_off = off;
            off += lds_level_bytes(Lv.G, c->ne, c->nc, c->f32 ? 4 : 8);
        }
    }
}

// Record the two coarse programs of context c from level c->lc (with the
// LDS plan c->l_lds) and upload the operation list.  fits: the coarsest level
// has a thread per cell (merged runs allowed); reg_ok: level lc's half sweeps
// may run register-resident with the exchange area at LDS byte rs_off.
int record_coarse(nmg_ctx *c, bool fits, bool reg_ok, long rs_off)
{
    Level saved[16];
    for (int l = 0; l <= c->NL; ++l) saved[l] = c->L[l];
    c->rec.clear();
    int rc = NMG_OK;
    // The program: all consecutive calls of cycle(lc) that cycle(lc - 1)
    // makes (gamma of them, one when lc - 1 is the finest level), from a
    // zero correction, then level lc's correction materialized.  Runs of half
    // sweeps continue across the calls (the repeated colour at the junction
    // is elided as in the level-by-level launches).
    c->recording = true;
    set_zero(c, c->lc);
    const int calls = (c->lc == 1) ? 1 : c->prm.gamma;
    for (int g = 0; g < calls && !rc; ++g) rc = cycle(c, c->lc);
    if (!rc) rc = materialize(c, c->lc);
    c->recording = false;
    c->prog_len = (int)c->rec.size();
    for (int l = 0; l <= c->NL; ++l) c->L[l] = saved[l];
    if (rc) return rc;
    if (c->prog_len > kMaxCoarseOps) {
        c->lc = -1;                              // too long: per-level launches
        c->rec.clear();
        c->prog_len = 0;
        return NMG_OK;
    }
    merge_runs(c, fits);
    merge_reg_runs(c, reg_ok, rs_off);
    size_t ob = sizeof(CoarseOp) * c->rec.size();
    if (hipMalloc(&c->d_ops, ob) != hipSuccess) return fail(c, NMG_ENOMEM, "coarse-cycle program");
    HIPCHK(c, hipMemcpy(c->d_ops, c->rec.data(), ob, hipMemcpyHostToDevice));
    return NMG_OK;
}

int plan_coarse(nmg_ctx *c)
{
    c->lc = first_coarse_level(c);
    if (c->lc < 0) return NMG_OK;
    c->l_lds = lds_first_level(c, c->lc);
    const long rs_off = (lds_levels_bytes(c, c->l_lds) + 15) / 16 * 16;
    int rc = record_coarse(c, 2 * c->L[c->NL].G.plane <= kCoarseBlock,
                           reg_run_fits(c, c->lc, c->l_lds, rs_off), rs_off);
    if (rc || c->lc < 0) return rc;
    LevelDev lv[kMaxLevels];
    coarse_level_table(c, c->l_lds, lv);
    if (hipMalloc(&c->d_lv, sizeof lv) != hipSuccess) return fail(c, NMG_ENOMEM, "coarse-cycle tables");
    HIPCHK(c, hipMemcpy(c->d_lv, lv, sizeof lv, hipMemcpyHostToDevice));
    return NMG_OK;
}

int reduce_to_host(nmg_ctx *c, int nparts, double *out)
{
    HIPCHK(c, launch_reduce(c->partial, nparts, c->scal, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->h_scal, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *out = c->h_scal[0];
    return NMG_OK;
}

int assemble(nmg_ctx *c, const double *z, const double *U, double *R_out, double *res)
{
    Level &L0 = c->L[0];
    HIPCHK(c, launch_isolated(c->P, z, U, c->iso, c->stream));
    HIPCHK(c, launch_assemble(c->P, L0.G, z, U, c->iso, L0.A, L0.b, c->f32, R_out, c->partial,
                              c->stream));
    int rc = phase_mark(c, NMG_PHASE_ASSEMBLY);
    if (!rc) rc = build_coarse(c);
    if (!rc) rc = phase_mark(c, NMG_PHASE_GALERKIN);
    if (rc) return rc;
    if (res) {
        if ((rc = reduce_to_host(c, nblocks(cells(L0.G)), res))) return rc;
        return phase_mark(c, NMG_PHASE_NORM);
    }
    return NMG_OK;
}

// l1 norm of level 0's linear residual b - A x (synchronizes).
int level0_residual_norm(nmg_ctx *c, double *out)
{
    Level &L0 = c->L[0];
    HIPCHK(c, launch_lin_res_norm(c->dim, c->f32, L0.G, L0.A, L0.b, L0.x, c->partial, c->stream));
    return reduce_to_host(c, nblocks(cells(L0.G)), out);
}

// ---- Krylov acceleration of the adjoint solve ------------------------------
// Right-preconditioned GMRES(m) on level 0's system A x = b (the transposed
// Newton matrix and the adjoint right-hand side), the preconditioner being
// one multigrid cycle from zero.  Classical Gram-Schmidt with one
// re-orthogonalization pass; Givens rotations on the host; the true residual
// is recomputed at each restart.  Stops when ||b - A x||_2 <= tol ||b - A x0||_2
// or after max_cycles preconditioner applications; x is left in L[0].x
// (materialized) and b in L[0].b.

int kbuffers(nmg_ctx *c, int m)
{
    if (c->km == m) return NMG_OK;
    for (double **q : {&c->kV, &c->kg, &c->kx, &c->kw, &c->kpart, &c->kdots, &c->kcoef}) {
        if (*q) (void)hipFree(*q);
        *q = nullptr;
    }
    if (c->h_k) (void)hipHostFree(c->h_k);
    c->h_k = nullptr;
    c->km = 0;
    const long n = 2L * c->nc * c->L[0].G.plane;
    const size_t vb = sizeof(double) * (size_t)n;
    bool ok = hipMalloc(&c->kV, vb * (m + 1)) == hipSuccess && hipMalloc(&c->kg, vb) == hipSuccess &&
              hipMalloc(&c->kx, vb) == hipSuccess && hipMalloc(&c->kw, vb) == hipSuccess &&
              hipMalloc(&c->kpart, sizeof(double) * (size_t)(m + 1) * nblocks(n)) == hipSuccess &&
              hipMalloc(&c->kdots, sizeof(double) * (m + 1)) == hipSuccess &&
              hipMalloc(&c->kcoef, sizeof(double) * (m + 1)) == hipSuccess &&
              hipHostMalloc(&c->h_k, sizeof(double) * (m + 1), hipHostMallocDefault) == hipSuccess;
    if (!ok) return fail(c, NMG_ENOMEM, "Krylov vectors");
    c->km = m;
    return NMG_OK;
}

// out[k] = <V_k, w>, k < nv, to the host (synchronizes).
int kdots(nmg_ctx *c, long n, const double *V, int nv, const double *w, double *out)
{
    HIPCHK(c, launch_multidot(n, V, n, nv, w, c->kpart, c->kdots, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->h_k, c->kdots, sizeof(double) * nv, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < nv; ++k) out[k] = c->h_k[k];
    return NMG_OK;
}

// w = a w - sum_k coef[k] V_k.
int kaxpy(nmg_ctx *c, long n, const double *V, int nv, const double *coef, double a, double *w)
{
    if (nv > 0) {
        HIPCHK(c, hipStreamSynchronize(c->stream));        // h_k is reused by the next transfer
        for (int k = 0; k < nv; ++k) c->h_k[k] = coef[k];
        HIPCHK(c, hipMemcpyAsync(c->kcoef, c->h_k, sizeof(double) * nv, hipMemcpyHostToDevice,
                                 c->stream));
    }
    HIPCHK(c, launch_multi_axpy(n, V, n, nv, c->kcoef, a, w, c->stream));
    return NMG_OK;
}

// x_out = M^-1 v: one multigrid cycle from zero on right-hand side v.
int kprecond(nmg_ctx *c, const double *v, long n)
{
    Level &L0 = c->L[0];
    HIPCHK(c, hipMemcpyAsync(L0.b, v, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
    set_zero(c, 0);
    int rc = cycle(c, 0);
    if (!rc) rc = materialize(c, 0);
    return rc;
}

int adjoint_gmres(nmg_ctx *c, int m, double tol, int max_cycles, int *cycles)
{
    int rc = kbuffers(c, m);
    if (rc) return rc;
    Level &L0 = c->L[0];
    const long n = 2L * c->nc * L0.G.plane;
    const size_t vb = sizeof(double) * (size_t)n;
    double *V = c->kV;
    HIPCHK(c, hipMemcpyAsync(c->kg, L0.b, vb, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->kx, L0.x, vb, hipMemcpyDeviceToDevice, c->stream));
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), sv(m + 1), y(m), h(m + 1),
        h2(m + 1);
    auto Hij = [&](int i, int j) -> double & { return H[(size_t)i * m + j]; };
    int k = 0;
    double beta = 0.0, beta0 = -1.0;
    for (;;) {
        HIPCHK(c, launch_lin_res_vec(c->dim, L0.G, (const double *)L0.A, c->kg, c->kx, V, c->stream));
        if ((rc = kdots(c, n, V, 1, V, &beta))) return rc;
        beta = std::sqrt(beta);
        if (beta0 < 0) beta0 = beta;
        if (beta <= tol * beta0 || beta == 0.0 || k >= max_cycles) break;
        if ((rc = kaxpy(c, n, V, 0, nullptr, 1.0 / beta, V))) return rc;
        std::fill(sv.begin(), sv.end(), 0.0);
        sv[0] = beta;
        int j = 0;
        bool done = false;
        for (; j < m && k < max_cycles && !done; ++j) {
            double *w = V + (long)(j + 1) * n;
            if ((rc = kprecond(c, V + (long)j * n, n))) return rc;
            ++k;
            HIPCHK(c, launch_apply(c->dim, L0.G, (const double *)L0.A, (const double *)L0.x, w,
                                   c->stream));
            if ((rc = kdots(c, n, V, j + 1, w, h.data()))) return rc;
            if ((rc = kaxpy(c, n, V, j + 1, h.data(), 1.0, w))) return rc;
            if ((rc = kdots(c, n, V, j + 1, w, h2.data()))) return rc;
            if ((rc = kaxpy(c, n, V, j + 1, h2.data(), 1.0, w))) return rc;
            for (int i = 0; i <= j; ++i) Hij(i, j) = h[i] + h2[i];
            double nrm = 0.0;
            if ((rc = kdots(c, n, w, 1, w, &nrm))) return rc;
            nrm = std::sqrt(nrm);
            Hij(j + 1, j) = nrm;
            for (int i = 0; i < j; ++i) {
                const double a = Hij(i, j), bb = Hij(i + 1, j);
                Hij(i, j) = cs[i] * a + sn[i] * bb;
                Hij(i + 1, j) = -sn[i] * a + cs[i] * bb;
            }
            const double a = Hij(j, j), bb = Hij(j + 1, j);
            const double d = std::hypot(a, bb);
            cs[j] = d > 0.0 ? a / d : 1.0;
            sn[j] = d > 0.0 ? bb / d : 0.0;
            Hij(j, j) = d;
            Hij(j + 1, j) = 0.0;
            sv[j + 1] = -sn[j] * sv[j];
            sv[j] = cs[j] * sv[j];
            if (nrm == 0.0 || std::fabs(sv[j + 1]) <= tol * beta0) done = true;
            else if ((rc = kaxpy(c, n, V, 0, nullptr, 1.0 / nrm, w))) return rc;
        }
        // y = H^-1 s on the j columns built, u = V y, x += M^-1 u
        for (int i = j - 1; i >= 0; --i) {
            double v = sv[i];
            for (int q = i + 1; q < j; ++q) v -= Hij(i, q) * y[q];
            y[i] = Hij(i, i) != 0.0 ? v / Hij(i, i) : 0.0;
        }
        for (int i = 0; i < j; ++i) y[i] = -y[i];
        HIPCHK(c, hipMemsetAsync(c->kw, 0, vb, c->stream));
        if ((rc = kaxpy(c, n, V, j, y.data(), 1.0, c->kw))) return rc;
        if ((rc = kprecond(c, c->kw, n))) return rc;
        ++k;
        const double minus_one = -1.0;
        if ((rc = kaxpy(c, n, (const double *)L0.x, 1, &minus_one, 1.0, c->kx))) return rc;
    }
    HIPCHK(c, hipMemcpyAsync(L0.x, c->kx, vb, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(L0.b, c->kg, vb, hipMemcpyDeviceToDevice, c->stream));
    L0.st[0] = L0.st[1] = ST_VALID;
    L0.last = -1;
    *cycles = k;
    return NMG_OK;
}

// Physics of the coarse mesh of level l (same domain, (nx, ny) >> l).
Phys level_phys(const nmg_ctx *c, int l)
{
    Phys P = c->P;
    P.nx = c->grid.nx >> l;
    P.ny = c->dim == 1 ? 1 : c->grid.ny >> l;
    if (c->dim == 2) {
        double dx = (c->grid.x1 - c->grid.x0) / P.nx, dy = (c->grid.y1 - c->grid.y0) / P.ny;
        P.elen[0] = P.elen[1] = dy;
        P.elen[2] = P.elen[3] = dx;
    }
    return P;
}

// Algorithm 1, Step 1 on U in place (see nmg_params); *sweeps = the BLU-SGS
// sweeps done over all levels, level_sweeps[l] (nullable) those on level l.
// Step 1's coarse beds and states (allocated with the context when
// eps_p > 0).
int alloc_step1(nmg_ctx *c)
{
    const int NL = c->NL, nc = c->nc;
    // level 1 is the largest coarse level; a half sweep launches at most 16
    // lanes per cell of one colour
    const size_t c1 = cells(c->L[1].G);
    const size_t nparts = (size_t)nblocks(16 * (long)c1);
    size_t tot = nc * c1 + nparts;
    for (int l = 1; l <= NL; ++l) tot += (size_t)(1 + nc) * cells(c->L[l].G);
    if (hipMalloc(&c->init_pool, sizeof(double) * tot) != hipSuccess)
        return fail(c, NMG_ENOMEM, "Step 1 levels");
    size_t off = 0;
    for (int l = 1; l <= NL; ++l) {
        c->zl[l] = c->init_pool + off; off += cells(c->L[l].G);
        c->Ul[l] = c->init_pool + off; off += (size_t)nc * cells(c->L[l].G);
    }
    c->init_red = c->init_pool + off; off += nc * c1;
    c->init_part = c->init_pool + off;
    return NMG_OK;
}

// Most sweeps of Step 1 enqueued between two looks at the stop flag (even:
// every run starts at an even sweep index, see step1_sweeps).
constexpr int kStep1Ahead = 64;

// The three launches of `n` Step 1 sweeps on level l (see nested_init); the
// first sweep's index on the level is even.
int step1_sweeps(nmg_ctx *c, int l, int n, hipStream_t s)
{
    const Phys P = level_phys(c, l);
    const int lanes = c->blu_lanes;
    const double *zl = c->zl[l];
    double *Ul = c->Ul[l], *red = c->init_red;
    int *ctrl = reinterpret_cast<int *>(c->scal + 1);
    for (int k = 0; k < n; ++k) {
        StopTest test;
        test.partial = c->init_part;
        test.n = blu_half_blocks(P, lanes);
        test.parity = k & 1;
        test.max_sweeps = c->prm.init_max_sweeps;
        test.thr = std::ldexp(c->prm.eps_p, -l);
        test.ctrl = ctrl;
        HIPCHK(c, launch_blu_half_io(P, zl, Ul, Ul, red, 0, 1, lanes, s, ctrl, StopTest(),
                                     c->init_part));
        HIPCHK(c, launch_blu_half_io(P, zl, Ul, red, Ul, 1, 2, lanes, s, ctrl, test, nullptr));
        HIPCHK(c, launch_blu_half_io(P, zl, red, Ul, Ul, 0, 1, lanes, s, ctrl, StopTest(),
                                     nullptr));
    }
    return NMG_OK;
}

// A run of kStep1Ahead sweeps on level l as a graph, captured on a stream of
// its own the first time it is needed (its launches' arguments are the same
// for every run of the level and every solve of the context).
int step1_graph(nmg_ctx *c, int l, hipGraphExec_t *out)
{
    if (c->init_graph[l]) {
        *out = c->init_graph[l];
        return NMG_OK;
    }
    if (!c->cap_stream)
        HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = step1_sweeps(c, l, kStep1Ahead, c->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    HIPCHK(c, e);
    e = hipGraphInstantiate(&c->init_graph[l], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(c, e);
    *out = c->init_graph[l];
    return NMG_OK;
}

int nested_init(nmg_ctx *c, const double *z, double *U, int *sweeps, int *level_sweeps)
{
    const int NL = c->NL, nc = c->nc;
    *sweeps = 0;
    if (level_sweeps)
        for (int l = 0; l < kMaxLevels; ++l) level_sweeps[l] = 0;
    if (!(c->prm.eps_p > 0.0) || NL < 1) return NMG_OK;
    if (!c->init_pool) return fail(c, NMG_EINVAL, "Step 1 levels not allocated");
    const double *zp = z;
    const double *Up = U;
    for (int l = 1; l <= NL; ++l) {
        const LevelGeom &Gf = c->L[l - 1].G;
        HIPCHK(c, launch_average(c->dim, Gf.nx, Gf.ny, 1, zp, c->zl[l], c->stream));
        HIPCHK(c, launch_average(c->dim, Gf.nx, Gf.ny, nc, Up, c->Ul[l], c->stream));
        zp = c->zl[l];
        Up = c->Ul[l];
    }
    // On each level: residual, stop test (sum ||R_i||_1 < eps_p 2^-l or the
    // sweep cap), symmetric BLU-SGS sweep, repeated, in three launches per
    // sweep.  The first computes the residual norms of both colours at the
    // level's state (block partials) and the red half sweep from it, stored
    // to init_red so that the state stays as it was; the second does the
    // stop test on those partials before its stores and the two black half
    // sweeps, reading the red states from init_red; the third the last red
    // half sweep from init_red into the level's state.  The test sets a flag
    // that gates the launches behind it, so runs of sweeps are enqueued ahead
    // (2, 4, ... up to kStep1Ahead, the last run before the sweep cap cut to
    // end at it, rounded up to an even count) and the host reads the flag
    // once per run;
    // after the stop nothing is stored.  The sweeps performed are those of
    // the loop with the test on the host.  Runs of kStep1Ahead sweeps are
    // replayed from a graph per level (the sweep counter is on the device,
    // so the launches of every such run are the same), which spares the host
    // a launch call per kernel: on the small levels those calls took longer
    // than the kernels.
    int *ctrl = reinterpret_cast<int *>(c->scal + 1);
    int *h_ctrl = reinterpret_cast<int *>(c->h_scal + 1);
    for (int l = NL; l >= 1; --l) {
        HIPCHK(c, launch_step1_reset(ctrl, c->stream));
        int cnt = 0, rc;
        long queued = 0;    // sweeps enqueued on the level
        for (int ahead = 2;; ahead = std::min(2 * ahead, kStep1Ahead)) {
            // the test at sweep index init_max_sweeps stops for certain
            const long need = (long)c->prm.init_max_sweeps + 1 - queued;
            int n = (int)std::min<long>(ahead, std::max<long>(need, 1));
            n += n & 1;
            hipGraphExec_t g = nullptr;
            if (n == kStep1Ahead && c->step1_graph && step1_graph(c, l, &g) != NMG_OK) {
                // no graph (capture or instantiation refused): enqueue the
                // launches one by one from now on
                c->step1_graph = 0;
                c->err.clear();
                (void)hipGetLastError();
                g = nullptr;
            }
            if (g) {
                HIPCHK(c, hipGraphLaunch(g, c->stream));
            } else if ((rc = step1_sweeps(c, l, n, c->stream))) {
                return rc;
            }
            queued += n;
            HIPCHK(c, hipMemcpyAsync(h_ctrl, ctrl, 2 * sizeof(int), hipMemcpyDeviceToHost,
                                     c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            if (h_ctrl[0]) {
                cnt = h_ctrl[1];
                break;
            }
        }
        *sweeps += cnt;
        if (level_sweeps) level_sweeps[l] = cnt;
        const LevelGeom &Gf = c->L[l - 1].G;
        HIPCHK(c, launch_inject(c->dim, Gf.nx, Gf.ny, nc, c->Ul[l], l == 1 ? U : c->Ul[l - 1],
                                c->stream));
    }
    return NMG_OK;
}

int count_pinned(nmg_ctx *c, const double *z, const double *U, int *n)
{
    long N = cells(c->L[0].G);
    HIPCHK(c, launch_isolated(c->P, z, U, c->iso, c->stream));
    HIPCHK(c, launch_count_u8(c->iso, N, c->partial, c->stream));
    double v = 0;
    int rc = reduce_to_host(c, nblocks(N), &v);
    *n = (int)v;
    return rc;
}

int create_ctx(const nmg_grid *grid, const nmg_bc *bc, const nmg_params *params, void *stream,
               bool plan, nmg_ctx **out);

// Physics of the finest mesh for the kernels (validated arguments).
Phys make_phys(const nmg_grid *grid, const nmg_bc *bc, const nmg_params *params)
{
    Phys P;
    P.dim = grid->dim;
    P.nx = grid->nx;
    P.ny = grid->ny;
    P.flux = params->flux;
    P.dry_pin = params->dry_pin;
    P.g = params->g;
    P.alpha = params->alpha;
    P.eps = params->fd_eps;
    P.h_eps = params->h_eps;
    P.eps_r = params->eps_r;
    P.tau = params->tau;
    P.pos_theta = params->pos_theta;
    if (grid->dim == 1) {
        P.elen[0] = P.elen[1] = P.elen[2] = P.elen[3] = 1.0;
    } else {
        double dx = (grid->x1 - grid->x0) / grid->nx, dy = (grid->y1 - grid->y0) / grid->ny;
        P.elen[0] = P.elen[1] = dy;
        P.elen[2] = P.elen[3] = dx;
    }
    for (int f = 0; f < 4; ++f) {
        const nmg_side &s = bc->side[f];
        P.bc[f].kind = s.kind;
        P.bc[f].h = s.h;
        P.bc[f].qn = s.qn;
        P.bc[f].ut = s.ut;
        P.bc[f].hasq = !std::isnan(s.qn);
        P.bc[f].hash = !std::isnan(s.h);
        P.bc[f].hast = !std::isnan(s.ut);
    }
    return P;
}

}  // namespace

// ---------------------------------------------------------------------------
extern "C" {

int nmg_create(const nmg_grid *grid, const nmg_bc *bc, const nmg_params *params, void *stream,
               nmg_ctx **out)
{
    if (!out) return NMG_EINVAL;
    *out = nullptr;
    return create_ctx(grid, bc, params, stream, true, out);
}

}  // extern "C"

namespace {

int create_ctx(const nmg_grid *grid, const nmg_bc *bc, const nmg_params *params, void *stream,
               bool plan, nmg_ctx **out)
{
    std::string msg;
    int rc = check_params(grid, bc, params, msg);
    if (rc) return rc;
    nmg_ctx *c = new (std::nothrow) nmg_ctx();
    if (!c) return NMG_ENOMEM;
    c->grid = *grid;
    c->bc = *bc;
    c->prm = *params;
    c->stream = (hipStream_t)stream;
    c->dim = grid->dim;
    c->nc = grid->dim == 1 ? 2 : 3;
    c->nb = grid->dim == 1 ? 3 : 5;
    c->ne = c->nb * c->nc * c->nc;
    c->NL = params->n_levels;

    c->P = make_phys(grid, bc, params);

    c->f32 = params->inner_fp32 != 0;
    if (const char *e = std::getenv("NMG_FUSE")) c->fuse = std::atoi(e);
    if (const char *e = std::getenv("NMG_COARSE_SPLIT")) c->split = std::atoi(e) != 0;
    if (const char *e = std::getenv("NMG_BLU_LANES")) {
        const int v = std::atoi(e);
        c->blu_lanes = (v == 1 || v == 4 || v == 16) ? v : -1;
    }
    if (const char *e = std::getenv("NMG_STEP1_GRAPH")) c->step1_graph = std::atoi(e) != 0;
    const size_t esz = c->f32 ? sizeof(float) : sizeof(double);
    size_t total = 0;   // elements
    for (int l = 0; l <= c->NL; ++l) {
        int nx = grid->nx >> l, ny = grid->dim == 1 ? 1 : grid->ny >> l;
        c->L[l].G = make_geom(nx, ny);
        total += (size_t)2 * c->ne * c->L[l].G.planeP + (size_t)2 * 2 * c->nc * c->L[l].G.plane +
                 (l > 0 ? (size_t)c->nc * c->L[l].G.plane : 0);
    }
    if (plan) total += (size_t)c->nc * c->L[0].G.plane;      // rres (not used by batches)
    char *pool = nullptr;
    if (hipMalloc(&pool, total * esz) != hipSuccess) {
        delete c;
        return NMG_ENOMEM;
    }
    c->pool = pool;
    size_t off = 0;
    for (int l = 0; l <= c->NL; ++l) {
        Level &Lv = c->L[l];
        Lv.A = pool + off * esz; off += (size_t)2 * c->ne * Lv.G.planeP;
        Lv.b = pool + off * esz; off += (size_t)2 * c->nc * Lv.G.plane;
        Lv.x = pool + off * esz; off += (size_t)2 * c->nc * Lv.G.plane;
        if (l > 0) {      // fused pairs never run on the finest level
            Lv.xt = pool + off * esz;
            off += (size_t)c->nc * Lv.G.plane;
        }
    }
    if (plan) {
        c->rres = pool + off * esz;
        off += (size_t)c->nc * c->L[0].G.plane;
    }
    long N = cells(c->L[0].G);
    int nparts = nblocks(N);
    bool ok = hipMemsetAsync(pool, 0, total * esz, c->stream) == hipSuccess &&
              (!(params->eps_p > 0.0) || c->NL < 1 || alloc_step1(c) == NMG_OK) &&
              hipMalloc(&c->iso, N) == hipSuccess &&
              hipMalloc(&c->partial, sizeof(double) * (nparts + 1)) == hipSuccess &&
              hipMalloc(&c->scal, sizeof(double) * 4) == hipSuccess &&
              hipHostMalloc(&c->h_scal, sizeof(double) * 4, hipHostMallocDefault) == hipSuccess &&
              hipMalloc(&c->Ulast, sizeof(double) * c->nc * N) == hipSuccess;
    if (!ok) {
        nmg_destroy(c);
        return NMG_ENOMEM;
    }
    rc = plan ? plan_coarse(c) : NMG_OK;
    if (rc) {
        nmg_destroy(c);
        return rc;
    }
    *out = c;
    return NMG_OK;
}

}  // namespace

extern "C" {

void nmg_destroy(nmg_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto &e : c->ev) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    for (hipEvent_t e : c->pev) (void)hipEventDestroy(e);
    for (hipGraphExec_t g : c->init_graph)
        if (g) (void)hipGraphExecDestroy(g);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->pool) (void)hipFree(c->pool);
    if (c->At_alloc) (void)hipFree(c->At_alloc);
    for (double *q : {c->kV, c->kg, c->kx, c->kw, c->kpart, c->kdots, c->kcoef})
        if (q) (void)hipFree(q);
    if (c->h_k) (void)hipHostFree(c->h_k);
    if (c->init_pool) (void)hipFree(c->init_pool);
    if (c->iso) (void)hipFree(c->iso);
    if (c->partial) (void)hipFree(c->partial);
    if (c->scal) (void)hipFree(c->scal);
    if (c->h_scal) (void)hipHostFree(c->h_scal);
    if (c->Ulast) (void)hipFree(c->Ulast);
    if (c->d_ops) (void)hipFree(c->d_ops);
    if (c->d_lv) (void)hipFree(c->d_lv);
    delete c;
}

const char *nmg_last_error(const nmg_ctx *c) { return c ? c->err.c_str() : "null context"; }

int nmg_residual(nmg_ctx *c, const double *z, const double *U, double *R_out, double *res_l1_host)
{
    if (!c) return NMG_EINVAL;
    if (!z || !U) return fail(c, NMG_EINVAL, "null z or U");
    HIPCHK(c, launch_residual(c->P, z, U, R_out, c->partial, c->stream));
    if (res_l1_host) return reduce_to_host(c, nblocks(cells(c->L[0].G)), res_l1_host);
    return NMG_OK;
}

int nmg_assemble_residual_jacobian(nmg_ctx *c, const double *z, const double *U, double *R_out,
                                   double *res_l1_host)
{
    if (!c) return NMG_EINVAL;
    if (!z || !U) return fail(c, NMG_EINVAL, "null z or U");
    return assemble(c, z, U, R_out, res_l1_host);
}

int nmg_mg_vcycle(nmg_ctx *c, double *dU, int n_cycles)
{
    if (!c) return NMG_EINVAL;
    if (!dU || n_cycles < 0) return fail(c, NMG_EINVAL, "null dU or negative cycle count");
    Level &L0 = c->L[0];
    HIPCHK(c, launch_vec_to_split(c->nc, c->f32, L0.G, dU, L0.x, c->stream));
    L0.st[0] = L0.st[1] = ST_VALID;
    L0.last = -1;
    for (int k = 0; k < n_cycles; ++k) {
        int rc = cycle(c, 0);
        if (rc) return rc;
    }
    int rc = materialize(c, 0);
    if (rc) return rc;
    HIPCHK(c, launch_vec_from_split(c->nc, c->f32, L0.G, L0.x, dU, c->stream));
    return NMG_OK;
}

int nmg_sgs(nmg_ctx *c, int level, double *dU, int iters)
{
    if (!c) return NMG_EINVAL;
    if (!dU || iters < 0 || level < 0 || level > c->NL)
        return fail(c, NMG_EINVAL, "bad level, dU or iteration count");
    Level &Lv = c->L[level];
    HIPCHK(c, launch_vec_to_split(c->nc, c->f32, Lv.G, dU, Lv.x, c->stream));
    Lv.st[0] = Lv.st[1] = ST_VALID;
    Lv.last = -1;
    int rc = smooth(c, level, iters);
    if (rc) return rc;
    HIPCHK(c, launch_vec_from_split(c->nc, c->f32, Lv.G, Lv.x, dU, c->stream));
    return NMG_OK;
}

int nmg_blu_sweep(nmg_ctx *c, const double *z, double *U)
{
    if (!c) return NMG_EINVAL;
    if (!z || !U) return fail(c, NMG_EINVAL, "null z or U");
    HIPCHK(c, launch_blu_sweeps(c->P, z, U, 1, c->blu_lanes, c->stream));
    return NMG_OK;
}

int nmg_load_system(nmg_ctx *c, const double *A0, const double *b0)
{
    if (!c) return NMG_EINVAL;
    if (!A0 || !b0) return fail(c, NMG_EINVAL, "null A0 or b0");
    Level &L0 = c->L[0];
    HIPCHK(c, launch_mat_to_split(c->ne, c->f32, L0.G, A0, L0.A, c->stream));
    HIPCHK(c, launch_vec_to_split(c->nc, c->f32, L0.G, b0, L0.b, c->stream));
    return build_coarse(c);
}

int nmg_get_system(nmg_ctx *c, int level, double *A, double *b)
{
    if (!c) return NMG_EINVAL;
    if (level < 0 || level > c->NL) return fail(c, NMG_EINVAL, "level out of range");
    Level &Lv = c->L[level];
    if (A) HIPCHK(c, launch_mat_from_split(c->ne, c->f32, Lv.G, Lv.A, A, c->stream));
    if (b) HIPCHK(c, launch_vec_from_split(c->nc, c->f32, Lv.G, Lv.b, b, c->stream));
    return NMG_OK;
}

int nmg_newton_mg_solve(nmg_ctx *c, const double *z, double *U, double tol, nmg_stats *st)
{
    if (!c) return NMG_EINVAL;
    if (!z || !U) return fail(c, NMG_EINVAL, "null z or U");
    const nmg_params &p = c->prm;
    Level &L0 = c->L[0];
    const long N = cells(L0.G);
    const size_t vbytes = sizeof(double) * c->nc * N;
    int status = NMG_NOT_CONVERGED, n = 0, rc;
    double res = 0.0, res0 = 0.0;
    if ((rc = phase_mark(c, -1))) return rc;
    HIPCHK(c, launch_threshold(c->P, U, c->stream));
    int init_sweeps = 0;
    if ((rc = nested_init(c, z, U, &init_sweeps, st ? st->init_level_sweeps : nullptr)))
        return rc;                                                  // Step 1 (eps_p > 0)
    if ((rc = phase_mark(c, NMG_PHASE_STEP1))) return rc;
    for (n = 0; n < p.max_newton; ++n) {
        HIPCHK(c, hipMemcpyAsync(c->Ulast, U, vbytes, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, launch_blu_sweeps(c->P, z, U, p.blu_sweeps, c->blu_lanes, c->stream));
        if ((rc = phase_mark(c, NMG_PHASE_BLU))) return rc;
        if ((rc = assemble(c, z, U, nullptr, &res))) return rc;
        if (st && st->res_hist && n < st->hist_cap) st->res_hist[n] = res;
        if (n == 0) res0 = res;
        if (!std::isfinite(res)) {
            HIPCHK(c, hipMemcpyAsync(U, c->Ulast, vbytes, hipMemcpyDeviceToDevice, c->stream));
            status = NMG_ENONFINITE;
            break;
        }
        if (res < tol) { status = NMG_OK; break; }
        if (res > 1e8 * res0) { status = NMG_EDIVERGED; break; }
        set_zero(c, 0);
        for (int m = 0; m < p.n_mg; ++m)
            if ((rc = cycle(c, 0))) return rc;
        if ((rc = phase_mark(c, NMG_PHASE_CYCLES))) return rc;
        if ((rc = materialize(c, 0))) return rc;
        HIPCHK(c, launch_update(c->P, L0.G, L0.x, c->f32, U, c->stream));
        if ((rc = phase_mark(c, NMG_PHASE_UPDATE))) return rc;
    }
    if (status == NMG_NOT_CONVERGED) {
        HIPCHK(c, launch_residual(c->P, z, U, nullptr, c->partial, c->stream));
        if ((rc = reduce_to_host(c, nblocks(N), &res))) return rc;
    }
    if (st) {
        int np = 0;
        if ((rc = count_pinned(c, z, U, &np))) return rc;
        st->n_pinned = np;
        st->newton_steps = n;
        st->status = status;
        st->res_l1 = res;
        st->init_sweeps = init_sweeps;
    }
    if ((rc = phase_mark(c, NMG_PHASE_FINAL))) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return status;
}

int nmg_adjoint_solve(nmg_ctx *c, const double *z, const double *U, const double *g,
                      double *lambda, double tol, int max_cycles, int krylov, int *cycles_host,
                      double *rel_res_host)
{
    if (!c) return NMG_EINVAL;
    if (!z || !U || !g || !lambda) return fail(c, NMG_EINVAL, "null z, U, g or lambda");
    if (max_cycles < 0 || !(tol >= 0)) return fail(c, NMG_EINVAL, "bad tol or max_cycles");
    if (krylov < 0 || krylov > 200) return fail(c, NMG_EINVAL, "krylov restart out of range");
    if (krylov > 0 && c->f32) return fail(c, NMG_EINVAL, "Krylov acceleration needs the FP64 hierarchy");
    Level &L0 = c->L[0];
    const size_t mbytes = (size_t)2 * c->ne * L0.G.planeP * (c->f32 ? sizeof(float) : sizeof(double));
    if (!c->At_alloc) {
        if (hipMalloc(&c->At_alloc, mbytes) != hipSuccess) return fail(c, NMG_ENOMEM, "adjoint matrix");
        c->At_spare = c->At_alloc;
    }
    HIPCHK(c, launch_isolated(c->P, z, U, c->iso, c->stream));
    HIPCHK(c, launch_assemble(c->P, L0.G, z, U, c->iso, L0.A, L0.b, c->f32, nullptr, c->partial,
                              c->stream));
    HIPCHK(c, launch_transpose(c->dim, c->f32, L0.G, L0.A, c->At_spare, c->stream));
    std::swap(L0.A, c->At_spare);
    int rc = build_coarse(c);
    if (rc) return rc;
    HIPCHK(c, launch_vec_to_split(c->nc, c->f32, L0.G, g, L0.b, c->stream));
    HIPCHK(c, launch_vec_to_split(c->nc, c->f32, L0.G, lambda, L0.x, c->stream));
    L0.st[0] = L0.st[1] = ST_VALID;
    L0.last = -1;
    double r0 = 0.0, r = 0.0;
    if ((rc = level0_residual_norm(c, &r0))) return rc;
    r = r0;
    int k = 0;
    if (krylov == 0) {
        // stationary iteration: multigrid cycles on A^T lambda = g
        while (k < max_cycles && r > tol * r0) {
            if ((rc = cycle(c, 0))) return rc;
            if ((rc = materialize(c, 0))) return rc;
            ++k;
            if ((rc = level0_residual_norm(c, &r))) return rc;
        }
    } else if (r0 > 0.0) {
        if ((rc = adjoint_gmres(c, krylov, tol, max_cycles, &k))) return rc;
        if ((rc = level0_residual_norm(c, &r))) return rc;
    }
    HIPCHK(c, launch_vec_from_split(c->nc, c->f32, L0.G, L0.x, lambda, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (cycles_host) *cycles_host = k;
    if (rel_res_host) *rel_res_host = r0 > 0.0 ? r / r0 : 0.0;
    return NMG_OK;
}

int nmg_bed_vjp(nmg_ctx *c, const double *z, const double *U, const double *lambda, double *out)
{
    if (!c) return NMG_EINVAL;
    if (!z || !U || !lambda || !out) return fail(c, NMG_EINVAL, "null z, U, lambda or out");
    HIPCHK(c, launch_isolated(c->P, z, U, c->iso, c->stream));
    HIPCHK(c, launch_bed_vjp(c->P, z, U, c->iso, lambda, out, c->stream));
    return NMG_OK;
}

int nmg_timing_enable(nmg_ctx *c, int enable, int cap)
{
    if (!c) return NMG_EINVAL;
    if (enable) {
        if (cap < 0 || cap > (1 << 20)) return fail(c, NMG_EINVAL, "timing cap out of range");
        HIPCHK(c, hipStreamSynchronize(c->stream));
        while ((int)c->ev.size() < cap) {
            hipEvent_t a, b;
            HIPCHK(c, hipEventCreate(&a));
            if (hipEventCreate(&b) != hipSuccess) {
                (void)hipEventDestroy(a);
                return fail(c, NMG_EHIP, "hipEventCreate failed");
            }
            c->ev.emplace_back(a, b);
        }
        c->ev_cells.assign(c->ev.size(), 0);
        c->ev_launches.assign(c->ev.size(), 0);
        c->nrec = 0;
        c->tgroup = -1;
        while ((int)c->pev.size() < cap) {
            hipEvent_t a;
            HIPCHK(c, hipEventCreate(&a));
            c->pev.push_back(a);
        }
        c->pev_ph.assign(c->pev.size(), -1);
        c->npev = 0;
    }
    c->timing = enable != 0;
    return NMG_OK;
}

int nmg_timing_read(nmg_ctx *c, double *ms_host, int *launches_host, long long *cells_host)
{
    if (!c) return NMG_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double tot = 0.0;
    long long cl = 0;
    int nl = 0;
    for (int k = 0; k < c->nrec; ++k) {
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev[k].first, c->ev[k].second));
        tot += ms;
        cl += c->ev_cells[k];
        nl += c->ev_launches[k];
    }
    if (ms_host) *ms_host = tot;
    if (launches_host) *launches_host = nl;
    if (cells_host) *cells_host = cl;
    return NMG_OK;
}

int nmg_timing_phases(nmg_ctx *c, double *ms_host, int *marks_host)
{
    if (!c) return NMG_EINVAL;
    if (!ms_host) return fail(c, NMG_EINVAL, "null ms_host");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int q = 0; q < NMG_NPHASES; ++q) ms_host[q] = 0.0;
    for (int k = 1; k < c->npev; ++k) {
        const int ph = c->pev_ph[k];
        if (ph < 0) continue;
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->pev[k - 1], c->pev[k]));
        ms_host[ph] += ms;
    }
    if (marks_host) *marks_host = c->npev;
    return NMG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches of independent problems.  Every instance has its own hierarchy
// (its own context); the first instance's state machine issues each
// operation of Algorithm 0 and Algorithm 1 once, and each operation is one
// launch over a work list of (instance, tile) items covering every instance
// still iterating.  All instances share the solver parameters, so the
// sequence of operations is the same for each; the coarse-cycle kernel runs
// one workgroup per instance.

namespace {

int bfail(nmg_batch *b, int code, const std::string &msg)
{
    if (b) b->err = msg;
    return code;
}

#define BHIPCHK(b, call)                                                                    \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return bfail(b, NMG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)

// Error of the driving context (its state machine's launches) moved to the batch.
int bctx(nmg_batch *b, int rc)
{
    if (rc) b->err = b->inst[0]->err;
    return rc;
}

struct RangeBuilder {
    std::vector<WorkItem> items;
    std::vector<std::pair<WorkRange *, long>> refs;
    // For each instance k, ceil(units[k] / tile) consecutive items.
    void add(WorkRange *w, const std::vector<long> &units, int tile)
    {
        const long off = (long)items.size();
        for (size_t k = 0; k < units.size(); ++k) {
            const long nt = (units[k] + tile - 1) / tile;
            for (long t = 0; t < nt; ++t) items.push_back(WorkItem{(int)k, (int)t});
        }
        w->n = (int)((long)items.size() - off);
        refs.emplace_back(w, off);
    }
};

int upload_mask(nmg_batch *b, int *d, const int *h)
{
    BHIPCHK(b, hipMemcpyAsync(d, h, sizeof(int) * b->n, hipMemcpyHostToDevice, b->stream));
    return NMG_OK;
}

// Per-instance sums of the level-0 partials into h_norm (synchronizes).
int batch_norms(nmg_batch *b, const int *d_which)
{
    BHIPCHK(b, launch_b_reduce(b->d_partial, b->d_roff, b->d_rcnt, b->n, d_which, b->d_norm,
                               b->stream));
    BHIPCHK(b, hipMemcpyAsync(b->h_norm, b->d_norm, sizeof(double) * b->n, hipMemcpyDeviceToHost,
                              b->stream));
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    return NMG_OK;
}

}  // namespace

extern "C" {

int nmg_batch_create(int n, const nmg_grid *grids, const nmg_bc *bcs, const nmg_params *params,
                     void *stream, nmg_batch **out)
{
    if (!out) return NMG_EINVAL;
    *out = nullptr;
    if (n < 1 || n > 65536 || !grids || !bcs || !params) return NMG_EINVAL;
    if (params->eps_p != 0.0) return NMG_EINVAL;        // Step 1 is not batched
    for (int k = 1; k < n; ++k)
        if (grids[k].dim != grids[0].dim) return NMG_EINVAL;
    nmg_batch *b = new (std::nothrow) nmg_batch();
    if (!b) return NMG_ENOMEM;
    b->n = n;
    b->stream = (hipStream_t)stream;
    b->prm = *params;
    b->dim = grids[0].dim;
    b->nc = b->dim == 1 ? 2 : 3;
    b->NL = params->n_levels;
    b->f32 = params->inner_fp32 != 0;
    for (int l = 0; l < kMaxLevels; ++l) b->tile[l] = kBlock;
    // NMG_BATCH_PERSISTENT = k > 0: the half sweeps run on a persistent grid of
    // k blocks per compute unit (measured on the 64-channel batch, k = 1..8:
    // 1-9 % slower than one block per work item, which stays the default)
    if (const char *e = std::getenv("NMG_BATCH_PERSISTENT")) b->persist = std::max(0, std::atoi(e)) * 256;
    for (int k = 0; k < n; ++k) {
        nmg_ctx *c = nullptr;
        int rc = create_ctx(&grids[k], &bcs[k], params, stream, false, &c);
        if (rc) {
            nmg_batch_destroy(b);
            return rc;
        }
        b->inst.push_back(c);
    }
    nmg_ctx *t = b->inst[0];
    t->batch = b;
    const int NL = b->NL;
    auto geom = [&](int k, int l) -> const LevelGeom & { return b->inst[k]->L[l].G; };

    // one coarse plan for every instance: the first level where all have at
    // most the limit's cells, LDS levels that fit every instance
    t->lc = -1;
    const long maxcells = coarse_cells_limit();
    for (int l = 1; l <= NL && t->lc < 0; ++l) {
        bool all = true;
        for (int k = 0; k < n; ++k) all = all && cells(geom(k, l)) <= maxcells;
        if (all) t->lc = l;
    }
    if (t->lc >= 0) {
        int l_lds = -2;
        bool fits = true;
        for (int k = 0; k < n; ++k) {
            const int lk = lds_first_level(b->inst[k], t->lc);
            if (lk < 0) { l_lds = -1; break; }
            l_lds = lk > l_lds ? lk : l_lds;
        }
        for (int k = 0; k < n; ++k) fits = fits && 2 * geom(k, NL).plane <= kCoarseBlock;
        t->l_lds = l_lds < 0 ? -1 : l_lds;
        long rs_off = 0;
        for (int k = 0; k < n; ++k) {
            const long used = (lds_levels_bytes(b->inst[k], t->l_lds) + 15) / 16 * 16;
            rs_off = used > rs_off ? used : rs_off;
        }
        bool reg_ok = true;
        for (int k = 0; k < n; ++k) reg_ok = reg_ok && reg_run_fits(b->inst[k], t->lc, t->l_lds, rs_off);
        int rc = record_coarse(t, fits, reg_ok, rs_off);
        if (rc) {
            b->err = t->err;
            nmg_batch_destroy(b);
            return rc;
        }
    }
    if (t->lc >= 0) {
        std::vector<LevelDev> clv((size_t)n * kMaxLevels);
        for (int k = 0; k < n; ++k) coarse_level_table(b->inst[k], t->l_lds, &clv[(size_t)k * kMaxLevels]);
        if (hipMalloc(&b->d_clv, sizeof(LevelDev) * clv.size()) != hipSuccess) {
            nmg_batch_destroy(b);
            return NMG_ENOMEM;
        }
        if (hipMemcpy(b->d_clv, clv.data(), sizeof(LevelDev) * clv.size(), hipMemcpyHostToDevice) !=
            hipSuccess) {
            nmg_batch_destroy(b);
            return NMG_EHIP;
        }
    }

    // work lists
    RangeBuilder rb;
    std::vector<long> u(n);
    for (int k = 0; k < n; ++k) u[k] = cells(geom(k, 0));
    rb.add(&b->w_cells0, u, kBlock);
    std::vector<int> roff(n), rcnt(n);
    {
        long pos = 0;
        for (int k = 0; k < n; ++k) {
            roff[k] = (int)pos;
            rcnt[k] = (int)((u[k] + kBlock - 1) / kBlock);
            pos += rcnt[k];
        }
    }
    for (int l = 0; l <= NL; ++l) {
        for (int k = 0; k < n; ++k) u[k] = geom(k, l).plane;
        for (int ti = 0; ti < kNumTiles; ++ti) rb.add(&b->w_plane[l][ti], u, kTileChoices[ti]);
        if (l >= 1) {
            for (int k = 0; k < n; ++k) u[k] = cells(geom(k, l));
            rb.add(&b->w_ccells[l], u, kBlock);
            for (int k = 0; k < n; ++k) u[k] = cells(geom(k, l)) * (b->dim == 1 ? 2 : 4);
            rb.add(&b->w_rchild[l], u, kBlock);
            for (int k = 0; k < n; ++k)
                u[k] = (long)((geom(k, l).nx + kPairTX - 1) / kPairTX) *
                       ((geom(k, l).ny + kPairTY - 1) / kPairTY);
            rb.add(&b->w_tile2d[l], u, 1);
        }
        for (int k = 0; k < n; ++k) b->cells_l[l] += cells(geom(k, l));
    }
    // residual planes of the last pre-smoothing half sweep, one per instance
    const size_t esz = b->f32 ? sizeof(float) : sizeof(double);
    std::vector<size_t> rr_off(n);
    size_t rr_total = 0;
    for (int k = 0; k < n; ++k) {
        rr_off[k] = rr_total;
        rr_total += (size_t)b->nc * geom(k, 0).plane * esz;
    }
    if (hipMalloc(&b->d_rr, rr_total) != hipSuccess) {
        nmg_batch_destroy(b);
        return NMG_ENOMEM;
    }
    t->rres = b->d_rr;          // enables the batched residual half sweeps
    std::vector<BatchLevel> blv((size_t)(NL + 1) * n);
    for (int l = 0; l <= NL; ++l)
        for (int k = 0; k < n; ++k) {
            const Level &Lf = b->inst[k]->L[l];
            const Level &Lc = b->inst[k]->L[l < NL ? l + 1 : l];
            blv[(size_t)l * n + k] = BatchLevel{Lf.G, Lc.G, Lf.A, Lf.b, Lf.x, Lc.A, Lc.b, Lc.x,
                                                Lf.xt, (char *)b->d_rr + rr_off[k]};
        }
    b->h_inst.resize(n);
    for (int k = 0; k < n; ++k) {
        nmg_ctx *c = b->inst[k];
        b->h_inst[k] = BatchInst{c->P, c->L[0].G, nullptr, nullptr, c->Ulast, c->iso,
                                 c->L[0].A, c->L[0].b, c->L[0].x};
    }
    bool ok = hipMalloc(&b->d_work, sizeof(WorkItem) * rb.items.size()) == hipSuccess &&
              hipMalloc(&b->d_lv, sizeof(BatchLevel) * blv.size()) == hipSuccess &&
              hipMalloc(&b->d_inst, sizeof(BatchInst) * n) == hipSuccess &&
              hipMalloc(&b->d_active, sizeof(int) * n) == hipSuccess &&
              hipMalloc(&b->d_mask, sizeof(int) * n) == hipSuccess &&
              hipHostMalloc(&b->h_active, sizeof(int) * n, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&b->h_mask, sizeof(int) * n, hipHostMallocDefault) == hipSuccess &&
              hipMalloc(&b->d_roff, sizeof(int) * n) == hipSuccess &&
              hipMalloc(&b->d_rcnt, sizeof(int) * n) == hipSuccess &&
              hipMalloc(&b->d_partial, sizeof(double) * (b->w_cells0.n + 1)) == hipSuccess &&
              hipMalloc(&b->d_norm, sizeof(double) * n) == hipSuccess &&
              hipHostMalloc(&b->h_norm, sizeof(double) * n, hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        nmg_batch_destroy(b);
        return NMG_ENOMEM;
    }
    ok = hipMemcpy(b->d_work, rb.items.data(), sizeof(WorkItem) * rb.items.size(),
                   hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(b->d_lv, blv.data(), sizeof(BatchLevel) * blv.size(), hipMemcpyHostToDevice) ==
             hipSuccess &&
         hipMemcpy(b->d_roff, roff.data(), sizeof(int) * n, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(b->d_rcnt, rcnt.data(), sizeof(int) * n, hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        nmg_batch_destroy(b);
        return NMG_EHIP;
    }
    for (auto &r : rb.refs) r.first->items = b->d_work + r.second;
    for (int k = 0; k < n; ++k) b->h_active[k] = b->h_mask[k] = 1;
    *out = b;
    return NMG_OK;
}

void nmg_batch_destroy(nmg_batch *b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    for (nmg_ctx *c : b->inst) {
        c->batch = nullptr;
        nmg_destroy(c);
    }
    if (b->d_inst) (void)hipFree(b->d_inst);
    if (b->d_lv) (void)hipFree(b->d_lv);
    if (b->d_rr) (void)hipFree(b->d_rr);
    if (b->d_clv) (void)hipFree(b->d_clv);
    if (b->d_work) (void)hipFree(b->d_work);
    if (b->d_active) (void)hipFree(b->d_active);
    if (b->d_mask) (void)hipFree(b->d_mask);
    if (b->h_active) (void)hipHostFree(b->h_active);
    if (b->h_mask) (void)hipHostFree(b->h_mask);
    if (b->d_roff) (void)hipFree(b->d_roff);
    if (b->d_rcnt) (void)hipFree(b->d_rcnt);
    if (b->d_partial) (void)hipFree(b->d_partial);
    if (b->d_norm) (void)hipFree(b->d_norm);
    if (b->h_norm) (void)hipHostFree(b->h_norm);
    delete b;
}

const char *nmg_batch_last_error(const nmg_batch *b) { return b ? b->err.c_str() : "null batch"; }

int nmg_batch_autotune(nmg_batch *b, int reps, int *tiles_out)
{
    if (!b) return NMG_EINVAL;
    if (reps < 1 || reps > 1000) return bfail(b, NMG_EINVAL, "reps out of range");
    nmg_ctx *t = b->inst[0];
    for (int k = 0; k < b->n; ++k) b->h_active[k] = 1;
    int rc = upload_mask(b, b->d_active, b->h_active);
    if (rc) return rc;
    hipEvent_t e0, e1;
    BHIPCHK(b, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return bfail(b, NMG_EHIP, "hipEventCreate failed");
    }
    rc = NMG_OK;
    for (int l = 0; l <= b->NL && !rc; ++l) {
        b->tile[l] = kBlock;
        if (t->lc >= 0 && l >= t->lc) continue;      // runs inside the coarse-cycle kernel
        float best = 0.0f;
        for (int ti = 0; ti < kNumTiles && !rc; ++ti) {
            const BatchLevel *lv = b->d_lv + (long)l * b->n;
            auto sweep = [&]() {
                return launch_b_sgs_half(b->dim, b->f32, MODE_NORMAL, kTileChoices[ti], lv,
                                         b->w_plane[l][ti], b->d_active, 0, b->persist,
                                         b->stream);
            };
            float ms = 0.0f;
            if (sweep() != hipSuccess || hipEventRecord(e0, b->stream) != hipSuccess) { rc = NMG_EHIP; break; }
            for (int r = 0; r < reps && !rc; ++r)
                if (sweep() != hipSuccess) rc = NMG_EHIP;
            if (rc || hipEventRecord(e1, b->stream) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = NMG_EHIP;
                break;
            }
            if (ti == 0 || ms < best) {
                best = ms;
                b->tile[l] = kTileChoices[ti];
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return bfail(b, rc, "autotune launch failed");
    // the sweeps above changed the corrections: every cycle starts from zero
    for (int l = 0; l <= b->NL; ++l) set_zero(t, l);
    if (tiles_out)
        for (int l = 0; l <= b->NL; ++l) tiles_out[l] = b->tile[l];
    return NMG_OK;
}

int nmg_batch_newton_mg_solve(nmg_batch *b, const double *const *z, double *const *U, double tol,
                              nmg_stats *stats)
{
    if (!b) return NMG_EINVAL;
    if (!z || !U) return bfail(b, NMG_EINVAL, "null z or U array");
    const int n = b->n;
    for (int k = 0; k < n; ++k) {
        if (!z[k] || !U[k]) return bfail(b, NMG_EINVAL, "null z or U");
        b->h_inst[k].z = z[k];
        b->h_inst[k].U = U[k];
    }
    nmg_ctx *t = b->inst[0];
    const nmg_params &p = b->prm;
    const int dim = b->dim;
    BHIPCHK(b, hipMemcpyAsync(b->d_inst, b->h_inst.data(), sizeof(BatchInst) * n,
                              hipMemcpyHostToDevice, b->stream));
    for (int k = 0; k < n; ++k) b->h_active[k] = 1;
    int rc = upload_mask(b, b->d_active, b->h_active);
    if (rc) return rc;
    std::vector<int> status(n, NMG_NOT_CONVERGED), steps(n, 0);
    std::vector<double> res(n, 0.0), res0(n, 0.0);
    int nactive = n;
    BHIPCHK(b, launch_b_threshold(dim, b->d_inst, b->w_cells0, b->d_active, b->stream));
    int ti256 = 0;
    while (kTileChoices[ti256] != kBlock) ++ti256;
    int it = 0;
    for (it = 0; it < p.max_newton && nactive > 0; ++it) {
        BHIPCHK(b, launch_b_copy_state(dim, b->d_inst, b->w_cells0, b->d_active, 0, b->stream));
        const int order[4] = {0, 1, 1, 0};
        for (int s = 0; s < p.blu_sweeps; ++s)
            for (int q = 0; q < 4; ++q)
                BHIPCHK(b, launch_b_blu_half(dim, b->d_inst, b->w_plane[0][ti256], b->d_active,
                                             order[q], b->stream));
        BHIPCHK(b, launch_b_isolated(dim, b->d_inst, b->w_cells0, b->d_active, b->stream));
        BHIPCHK(b, launch_b_assemble(dim, b->f32, b->d_inst, b->w_cells0, b->d_active,
                                     b->d_partial, b->stream));
        if ((rc = bctx(b, build_coarse(t)))) return rc;
        if ((rc = batch_norms(b, b->d_active))) return rc;
        bool restore = false, changed = false;
        for (int k = 0; k < n; ++k) {
            b->h_mask[k] = 0;
            if (!b->h_active[k]) continue;
            const double r = b->h_norm[k];
            if (stats && stats[k].res_hist && it < stats[k].hist_cap) stats[k].res_hist[it] = r;
            if (it == 0) res0[k] = r;
            res[k] = r;
            int st = NMG_NOT_CONVERGED;
            bool done = true;
            if (!std::isfinite(r)) {
                st = NMG_ENONFINITE;
                b->h_mask[k] = 1;
                restore = true;
            } else if (r < tol) {
                st = NMG_OK;
            } else if (r > 1e8 * res0[k]) {
                st = NMG_EDIVERGED;
            } else {
                done = false;
            }
            if (done) {
                status[k] = st;
                steps[k] = it;
                b->h_active[k] = 0;
                --nactive;
                changed = true;
            }
        }
        if (restore) {
            if ((rc = upload_mask(b, b->d_mask, b->h_mask))) return rc;
            BHIPCHK(b, launch_b_copy_state(dim, b->d_inst, b->w_cells0, b->d_mask, 1, b->stream));
        }
        if (changed && (rc = upload_mask(b, b->d_active, b->h_active))) return rc;
        if (nactive == 0) break;
        set_zero(t, 0);
        for (int m = 0; m < p.n_mg; ++m)
            if ((rc = bctx(b, cycle(t, 0)))) return rc;
        if ((rc = bctx(b, materialize(t, 0)))) return rc;
        BHIPCHK(b, launch_b_update(dim, b->f32, b->d_inst, b->w_cells0, b->d_active, b->stream));
    }
    // instances that used every Newton step: residual of the final state
    if (nactive > 0) {
        for (int k = 0; k < n; ++k) {
            if (b->h_active[k]) steps[k] = p.max_newton;
            b->h_mask[k] = b->h_active[k];
        }
        if ((rc = upload_mask(b, b->d_mask, b->h_mask))) return rc;
        BHIPCHK(b, launch_b_residual(dim, b->d_inst, b->w_cells0, b->d_mask, b->d_partial, b->stream));
        if ((rc = batch_norms(b, b->d_mask))) return rc;
        for (int k = 0; k < n; ++k)
            if (b->h_mask[k]) res[k] = b->h_norm[k];
    }
    if (stats) {
        for (int k = 0; k < n; ++k) b->h_mask[k] = 1;
        if ((rc = upload_mask(b, b->d_mask, b->h_mask))) return rc;
        BHIPCHK(b, launch_b_isolated(dim, b->d_inst, b->w_cells0, b->d_mask, b->stream));
        BHIPCHK(b, launch_b_count_iso(b->d_inst, b->w_cells0, b->d_mask, b->d_partial, b->stream));
        if ((rc = batch_norms(b, b->d_mask))) return rc;
        for (int k = 0; k < n; ++k) {
            stats[k].n_pinned = (int)b->h_norm[k];
            stats[k].newton_steps = steps[k];
            stats[k].status = status[k];
            stats[k].res_l1 = res[k];
            stats[k].init_sweeps = 0;
            for (int l = 0; l < kMaxLevels; ++l) stats[k].init_level_sweeps[l] = 0;
        }
    }
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    for (int k = 0; k < n; ++k)
        if (status[k] != NMG_OK) return NMG_NOT_CONVERGED;
    return NMG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Residual without allocation.  The block partial sums of the norm live in a
// file-scope device array of fixed size (every GPU the library runs on holds
// its own copy until the process ends); its device address is looked up
// once per device with that device current and kept, because in host code
// the array's name is not a device address.

namespace {

constexpr long kNoAllocMaxCells = 1L << 26;                 // 8192 x 8192
constexpr int kNoAllocParts = (int)(kNoAllocMaxCells / kBlock);   // 262,144 partials: 2 MiB

__device__ __align__(256) static double scratch[kNoAllocParts + 1];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (nullptr on failure).
double *scratch_on_current_device()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" int nmg_residual_noalloc(const nmg_grid *grid, const nmg_bc *bc,
                                    const nmg_params *params, void *stream, const double *z,
                                    const double *U, double *R_out, double *res_l1)
{
    std::string msg;
    if (check_params(grid, bc, params, msg)) return NMG_EINVAL;
    if (!z || !U) return NMG_EINVAL;
    const long N = (long)grid->nx * grid->ny;
    if (N > kNoAllocMaxCells) return NMG_EINVAL;
    double *part = scratch_on_current_device();
    if (!part) return NMG_EHIP;
    const Phys P = make_phys(grid, bc, params);
    hipStream_t s = (hipStream_t)stream;
    // every block of the residual writes its partial, and the reduction
    // reads exactly those, so nothing in the array needs clearing
    if (launch_residual(P, z, U, R_out, part, s) != hipSuccess) return NMG_EHIP;
    if (res_l1 && launch_reduce(part, nblocks(N), res_l1, s) != hipSuccess) return NMG_EHIP;
    return NMG_OK;
}
