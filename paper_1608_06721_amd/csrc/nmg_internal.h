// Internal interface between the host driver (nmg_api.hip) and the gfx950
// kernels (nmg_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>

namespace nmg {

// One side's boundary condition with its "prescribed" flags resolved.
struct SideDev {
    int kind;               // 0 reflect, 1 slip, 2 open
    int hasq, hash, hast;   // which of qn, h, ut are prescribed
    double h, qn, ut;
};

// Everything the discretization kernels need besides the arrays.
struct Phys {
    int dim, nx, ny;
    int flux, dry_pin;
    double g, alpha, eps, h_eps, eps_r, tau, pos_theta;
    double elen[4];         // |e| of W, E, S, N faces
    SideDev bc[4];
};

// Geometry of one multigrid level in the colour-split layout: every cell
// (i, j) lives in colour (i + j) & 1 at slot t = j * W + (i >> 1) of a
// [ny][W] plane, W = (nx + 1) / 2.  Vectors are [colour][NC][ny][W].
// Matrices are tiled by 64 slots (one wavefront): [colour][tile][NE][64],
// entry e = (block * NC + row) * NC + col, so the NE entries that one wave
// reads in a half sweep form one contiguous NE * 512-byte run.
constexpr int kTile = 64;

struct LevelGeom {
    int nx, ny, W;
    long plane;             // ny * W
    long planeP;            // plane rounded up to a multiple of kTile
};

inline LevelGeom make_geom(int nx, int ny)
{
    LevelGeom g;
    g.nx = nx;
    g.ny = ny;
    g.W = (nx + 1) / 2;
    g.plane = (long)ny * g.W;
    g.planeP = (g.plane + kTile - 1) / kTile * kTile;
    return g;
}

// Offset of entry 0 of slot t's block row in a colour-split tiled matrix
// with NE entries per row; entry e is at + e * kTile.
__host__ __device__ inline long mat_off(const LevelGeom &G, int NE, int color, long t)
{
    return (long)color * NE * G.planeP + (t / kTile) * NE * kTile + (t % kTile);
}

// Read mode of the other colour in a block SGS half sweep.
enum SweepMode {
    MODE_NORMAL = 0,        // other colour as stored
    MODE_ZERO = 1,          // other colour is zero (not materialized)
    MODE_PROLONG = 2,       // stored value + the parent's coarse correction
    MODE_PROLONG_ZERO = 3   // zero + the parent's coarse correction
};

constexpr int kBlock = 256;
constexpr int kPairTX = 32, kPairTY = 16;   // cell tiles of the fused half-sweep pairs
constexpr int kCoarseBlock = 512;     // one workgroup runs the coarse part of a cycle
constexpr int kMaxLevels = 16;
constexpr int kMaxCoarseOps = 1 << 16;  // longest recorded coarse program
// LDS bytes of the coarse-cycle kernel for level data: the coarsest levels
// whose blocks, block inverses and vectors fit are copied in and run from
// LDS (gfx950 allows 160 KB per workgroup; 16 bytes stay for a zero slot).
constexpr long kCoarseLdsBytes = 160 * 1024 - 16;

// Device-side description of one level (for the coarse-cycle kernel); the
// arrays hold the hierarchy's scalar type (double, or float for the FP32
// inner V-cycle).  lds_off >= 0: byte offset of the level's copy in the
// kernel's LDS (blocks, then block inverses, then b, then x); -1: the level
// is used in place in global memory.
struct LevelDev {
    LevelGeom G;
    void *A, *b, *x;
    long lds_off;
};

// One operation of the recorded coarse part of a cycle.  COP_RUN is count
// consecutive half sweeps of alternating colour on an LDS-resident level
// with a thread per cell, the first of them in `mode` (any start mode for
// COP_REGRUN, normal or zero start for COP_RUN) and the rest normal; for
// COP_RUN, aux = 1 allows two lanes per cell (3x3 blocks, where the level
// has at most kCoarseBlock / 4 cells per colour).
// COP_REGRUN is the same on a level in global memory with at most one slot
// per colour and thread, whose block rows stay in registers and whose x
// moves to the LDS bytes at lds_off for the run; aux = 1 appends the
// restriction to the next level, whose residuals are exchanged through the
// same LDS bytes.
enum CoarseOpKind { COP_SGS = 0, COP_RESTRICT = 1, COP_FIX = 2, COP_RUN = 3, COP_REGRUN = 4 };
struct CoarseOp {
    int kind;               // CoarseOpKind
    int level;
    int color;              // SGS / FIX: colour; RUN, REGRUN: colour of the first half sweep
    int mode;               // SGS / RUN / REGRUN: SweepMode; FIX: 0 zero, 1 add parent, 2 set parent
    int count;              // RUN, REGRUN: number of half sweeps
    int aux;                // REGRUN: 1 if the restriction follows; RUN: 1 allows two lanes per cell
    int lds_off;            // REGRUN: byte offset of the run's x / exchange area in LDS
};

inline int nblocks(long n) { return (int)((n + kBlock - 1) / kBlock); }

// A level whose block matrix is larger than this is fetched as read-once data
// (non-temporal hint) by its launched half sweeps and restriction; smaller
// levels are left to the caches, which serve their repeated visits in a
// cycle.  Measured on the 1024x1024 solve: streaming the finest level (377
// MB) gained 13% on its half sweep, adding the 512x512 level (94 MB) 1% on
// the solve, going down to 16 MB nothing more; streaming every level lost.
constexpr long kStreamBytes = 64L << 20;
inline bool stream_level(long cells, int nc, long elem_bytes)
{
    const long ne = (nc == 2 ? 3 : 5) * (long)nc * nc;
    return cells * ne * elem_bytes > kStreamBytes;
}

// ---- launchers (return hipError_t of the launch) ----
hipError_t launch_isolated(const Phys &P, const double *z, const double *U, unsigned char *iso,
                           hipStream_t s);
hipError_t launch_assemble(const Phys &P, const LevelGeom &G, const double *z, const double *U,
                           const unsigned char *iso, void *A, void *b, bool f32, double *R_out,
                           double *partial, hipStream_t s);
hipError_t launch_residual(const Phys &P, const double *z, const double *U, double *R_out,
                           double *partial, hipStream_t s);

// Reset of the Step 1 stop test's control words {stop flag, sweeps done,
// sweep counts by parity}.
hipError_t launch_step1_reset(int *ctrl, hipStream_t s);
hipError_t launch_reduce(const double *partial, int n, double *out, hipStream_t s);
hipError_t launch_count_u8(const unsigned char *v, long n, double *partial, hipStream_t s);
// lanes: lanes per cell, 1, 4 (k_blu_half_quad) or 16 (k_blu_half_x16, 2D;
// 4 in 1D), or -1 to choose by the mesh: 16 in 2D on meshes of at most
// kBluX16MaxCells cells per colour, 4 up to kBluQuadMaxCells, else 1.  Measured per half sweep, one
// lane against four per cell: 79 against 94 us with 524,288 cells per
// colour and 22 against 25 us with 131,072 (the arithmetic bounds these
// launches and four lanes repeat the cell's own side and block solve), 17
// against 10 us with 16,384 and 20-32 against 8-11 us on smaller levels
// (there a launch lasts as long as one cell's chain of dependent arithmetic).
constexpr long kBluQuadMaxCells = 1L << 16;
// 2D meshes of at most kBluX16MaxCells cells per colour run the half sweep
// with sixteen lanes per cell (k_blu_half_x16: one per face and evaluation).
constexpr long kBluX16MaxCells = 1L << 14;
// Step 1 stop test done by a BLU-SGS launch before its stores (no launch of
// its own): every block sums the n partials of the level's residual norm
// (written by the launch before it) in one fixed order, the same in every
// block, and the sweep stops if ctrl[0] is already set, the sum is below thr
// (or not a number), or the sweeps done on the level, ctrl[2 + parity], are
// max_sweeps.  Block 0 records a new stop (ctrl[0] = 1, ctrl[1] = sweeps
// done) or counts the sweep in ctrl[2 + (parity ^ 1)], the slot the next
// sweep reads, so no block reads a word that this launch writes.  parity:
// the sweep's index on the level mod 2.  partial == nullptr: no test.
struct StopTest {
    const double *partial = nullptr;
    int n = 0, parity = 0, max_sweeps = 0;
    double thr = 0.0;
    int *ctrl = nullptr;
};
// reps consecutive half sweeps of one colour in one launch (each cell
// updated reps times from its neighbours' unchanged states); gate: a stop
// flag set by an earlier launch, test: the stop test of this launch.
hipError_t launch_blu_half(const Phys &P, const double *z, double *U, int color, int reps,
                           int lanes, hipStream_t s, const int *gate = nullptr,
                           const StopTest &test = StopTest());
// The general form: own states read from Uown, the other colour's from
// Unb, new states stored to Uout; with res_partial (Uown == Unb) the launch
// also writes per block the sum of ||R_i||_1 at its input state over its
// slots' cells of both colours, blu_half_blocks(P, lanes) partials.
hipError_t launch_blu_half_io(const Phys &P, const double *z, const double *Uown,
                              const double *Unb, double *Uout, int color, int reps, int lanes,
                              hipStream_t s, const int *gate, const StopTest &test,
                              double *res_partial);
int blu_half_blocks(const Phys &P, int lanes);
// n symmetric BLU-SGS sweeps (half sweeps of colours 0, 1, 1, 0 each), runs
// of one colour merged into single launches: 0, 1 x2, 0 for one sweep.  The
// stop test, if any, is done by the first launch.
hipError_t launch_blu_sweeps(const Phys &P, const double *z, double *U, int n, int lanes,
                             hipStream_t s, const int *gate = nullptr,
                             const StopTest &test = StopTest());
hipError_t launch_update(const Phys &P, const LevelGeom &G, const void *x, bool f32, double *U,
                         hipStream_t s);
hipError_t launch_threshold(const Phys &P, double *U, hipStream_t s);

// Linear multigrid launchers; f32 selects the float hierarchy.
// stream: the level's matrix is fetched as read-once data (stream_level).
hipError_t launch_sgs_half(int dim, bool f32, int mode, const LevelGeom &G, const void *A,
                           const void *b, void *x, int color, const LevelGeom &Gc, const void *xc,
                           bool stream, hipStream_t s);
hipError_t launch_restrict(int dim, bool f32, const LevelGeom &G, const void *A, const void *b,
                           const void *x, const LevelGeom &Gc, void *bc, bool stream,
                           hipStream_t s);
// A normal-mode half sweep of colour `color` that also writes the updated
// cells' linear residuals to rout (NC planes of G.plane slots), and the
// restriction that takes the residuals of the children of colour rcol from
// rin instead of recomputing them (valid while both colours of x are as the
// half sweep left them).
hipError_t launch_sgs_half_res(int dim, bool f32, const LevelGeom &G, const void *A,
                               const void *b, void *x, int color, void *rout, bool stream,
                               hipStream_t s);
hipError_t launch_restrict_res(int dim, bool f32, const LevelGeom &G, const void *A,
                               const void *b, const void *x, const LevelGeom &Gc, void *bc,
                               const void *rin, int rcol, bool stream, hipStream_t s);
// Two consecutive half sweeps (colour `color` in `mode`, then the other colour
// in normal mode) in one launch, 2D only: colour `color` is updated in x, the
// other colour is read from xin (NC planes) and written to xout (NC planes).
hipError_t launch_sgs_pair(bool f32, int mode, const LevelGeom &G, const void *A, const void *b,
                           void *x, const void *xin, void *xout, int color, const LevelGeom &Gc,
                           const void *xc, hipStream_t s);
// Three consecutive half sweeps (colours color, other, color; the first in
// `mode`) in one launch, 2D only, with the buffers of launch_sgs_pair.
hipError_t launch_sgs_triple(bool f32, int mode, const LevelGeom &G, const void *A,
                             const void *b, void *x, const void *xin, void *xout, int color,
                             const LevelGeom &Gc, const void *xc, hipStream_t s);
hipError_t launch_galerkin(int dim, bool f32, const LevelGeom &Gf, const void *Af,
                           const LevelGeom &Gc, void *Ac, hipStream_t s);
// Materialize one colour of x: op 0 = set zero, 1 = add the parent's
// coarse value, 2 = set to the parent's coarse value.
hipError_t launch_fix_color(int dim, bool f32, int op, const LevelGeom &G, void *x, int color,
                            const LevelGeom &Gc, const void *xc, hipStream_t s);

// The recorded coarse part of a V-cycle, executed by one workgroup; levels
// l_lds..nl are staged in LDS (l_lds < 0: none).
hipError_t launch_coarse_cycle(int dim, bool f32, const CoarseOp *ops, int nops,
                               const LevelDev *lv, int l_lds, int nl, hipStream_t s);

// Sensitivities: block transpose of a level matrix (A and At distinct), the
// bed vector-Jacobian product (dR/dz)^T lam, and the l1 norm of a level's
// linear residual as per-block partial sums (nblocks(nx * ny) of them).
hipError_t launch_transpose(int dim, bool f32, const LevelGeom &G, const void *A, void *At,
                            hipStream_t s);
hipError_t launch_bed_vjp(const Phys &P, const double *z, const double *U,
                          const unsigned char *iso, const double *lam, double *out, hipStream_t s);
hipError_t launch_lin_res_norm(int dim, bool f32, const LevelGeom &G, const void *A,
                               const void *b, const void *x, double *partial, hipStream_t s);

// Level-0 vector operations of the Krylov-accelerated adjoint solve (FP64):
// y = A x; r = b - A x; out[k] = <V_k, w> for k < nv (V_k = V + k * ld,
// partial holds nv * nblocks(n) doubles); w = a w - sum_k c[k] V_k.
hipError_t launch_apply(int dim, const LevelGeom &G, const double *A, const double *x, double *y,
                        hipStream_t s);
hipError_t launch_lin_res_vec(int dim, const LevelGeom &G, const double *A, const double *b,
                              const double *x, double *r, hipStream_t s);
hipError_t launch_multidot(long n, const double *V, long ld, int nv, const double *w,
                           double *partial, double *out, hipStream_t s);
hipError_t launch_multi_axpy(long n, const double *V, long ld, int nv, const double *c, double a,
                             double *w, hipStream_t s);

// Algorithm 1, Step 1: child averages of ncomp planes of nxf x nyf fine cells
// onto the coarser mesh, and injection of a coarse state into the children.
hipError_t launch_average(int dim, int nxf, int nyf, int ncomp, const double *f, double *c,
                          hipStream_t s);
hipError_t launch_inject(int dim, int nxf, int nyf, int ncomp, const double *c, double *f,
                         hipStream_t s);

// ---- batches of independent problems -------------------------------------
// One instance of a batch at the Newton level.
struct BatchInst {
    Phys P;
    LevelGeom G0;               // level 0 of its hierarchy
    const double *z;
    double *U, *Ulast;
    unsigned char *iso;
    void *A, *b, *x;            // level-0 hierarchy arrays
};

// One instance of a batch at multigrid level l: the level, the next coarser
// level (the level itself at the coarsest) and their arrays.
struct BatchLevel {
    LevelGeom G, Gc;
    void *A, *b, *x;
    void *Ac, *bc, *xc;
    void *xt;               // the level's alternate planes for fused half-sweep pairs
    void *rr;               // the instance's residual planes (launch_b_sgs_half_res)
};

// One tile of one instance: a batched launch runs one block per work item.
struct WorkItem {
    int inst, tile;
};

// A contiguous range of a work list (the work items of one launch).
struct WorkRange {
    const WorkItem *items;
    int n;
};

// Tile lengths the batched half sweep can be launched with.
constexpr int kNumTiles = 4;
constexpr int kTileChoices[kNumTiles] = {64, 128, 256, 512};

// Batched launchers: every block handles one work item and skips instances
// whose active flag is 0.
hipError_t launch_b_isolated(int dim, const BatchInst *bi, WorkRange w, const int *active,
                             hipStream_t s);
hipError_t launch_b_assemble(int dim, bool f32, const BatchInst *bi, WorkRange w,
                             const int *active, double *partial, hipStream_t s);
hipError_t launch_b_residual(int dim, const BatchInst *bi, WorkRange w, const int *active,
                             double *partial, hipStream_t s);
hipError_t launch_b_count_iso(const BatchInst *bi, WorkRange w, const int *active,
                              double *partial, hipStream_t s);
// Per-instance sums of the partials: out[k] = sum of partial[off[k] .. off[k] + cnt[k])
// in the order of launch_reduce.
hipError_t launch_b_reduce(const double *partial, const int *off, const int *cnt, int n,
                           const int *active, double *out, hipStream_t s);
hipError_t launch_b_blu_half(int dim, const BatchInst *bi, WorkRange w, const int *active,
                             int color, hipStream_t s);
// Fused half-sweep pair of launch_sgs_pair over a work list of 32x16 tiles
// (2D): flip 0 reads the second colour from x and writes it to xt, flip 1
// the reverse.
hipError_t launch_b_sgs_pair(bool f32, int mode, const BatchLevel *lv, WorkRange w,
                             const int *active, int color, int flip, hipStream_t s);
hipError_t launch_b_update(int dim, bool f32, const BatchInst *bi, WorkRange w,
                           const int *active, hipStream_t s);
hipError_t launch_b_threshold(int dim, const BatchInst *bi, WorkRange w, const int *active,
                              hipStream_t s);
// dir 0: Ulast = U, dir 1: U = Ulast.
hipError_t launch_b_copy_state(int dim, const BatchInst *bi, WorkRange w, const int *active,
                               int dir, hipStream_t s);
// persist > 0: a persistent grid of that many blocks looping over the work
// list instead of one block per work item (kb_sgs_half_loop).
hipError_t launch_b_sgs_half(int dim, bool f32, int mode, int tile, const BatchLevel *lv,
                             WorkRange w, const int *active, int color, int persist,
                             hipStream_t s);
hipError_t launch_b_restrict(int dim, bool f32, const BatchLevel *lv, WorkRange w,
                             const int *active, hipStream_t s);
// Batched launch_sgs_half_res / launch_restrict_res (normal mode; each
// instance's residuals in its BatchLevel::rr).
hipError_t launch_b_sgs_half_res(int dim, bool f32, int tile, const BatchLevel *lv, WorkRange w,
                                 const int *active, int color, hipStream_t s);
hipError_t launch_b_restrict_res(int dim, bool f32, const BatchLevel *lv, WorkRange w,
                                 const int *active, int rcol, hipStream_t s);
hipError_t launch_b_fix_color(int dim, bool f32, int op, const BatchLevel *lv, WorkRange w,
                              const int *active, int color, hipStream_t s);
hipError_t launch_b_galerkin(int dim, bool f32, const BatchLevel *lv, WorkRange w,
                             const int *active, hipStream_t s);
// The coarse-cycle kernel with one workgroup per instance: workgroup k uses
// the level table lv + k * kMaxLevels and skips an inactive instance.
hipError_t launch_b_coarse_cycle(int dim, bool f32, const CoarseOp *ops, int nops,
                                 const LevelDev *lv, int ninst, const int *active, int l_lds,
                                 int nl, hipStream_t s);

// Bytes of one level's blocks, right-hand side and correction (both colours)
// for the scalar size esz.
inline long level_bytes(const LevelGeom &G, int ne, int nc, long esz)
{
    return (2 * ne * G.planeP + 2 * 2 * nc * G.plane) * esz;
}

// Entries of a block's precomputed inverse data: the NC x NC cofactors and
// the reciprocal determinant.
__host__ __device__ constexpr int inv_entries(int nc) { return nc * nc + 1; }

// Bytes of one level's LDS copy in the coarse-cycle kernel: level_bytes plus
// the block inverses of both colours, tiled like the blocks.
__host__ __device__ inline long lds_level_bytes(const LevelGeom &G, int ne, int nc, long esz)
{
    return (2 * ne * G.planeP + 2 * inv_entries(nc) * G.planeP + 2 * 2 * nc * G.plane) * esz;
}

// Layout conversions between the public FP64 layouts and the colour-split
// hierarchy storage.
hipError_t launch_vec_to_split(int nc, bool f32, const LevelGeom &G, const double *v, void *split,
                               hipStream_t s);
hipError_t launch_vec_from_split(int nc, bool f32, const LevelGeom &G, const void *split,
                                 double *v, hipStream_t s);
hipError_t launch_mat_to_split(int ne, bool f32, const LevelGeom &G, const double *A, void *split,
                               hipStream_t s);
hipError_t launch_mat_from_split(int ne, bool f32, const LevelGeom &G, const void *split,
                                 double *A, hipStream_t s);

}  // namespace nmg
