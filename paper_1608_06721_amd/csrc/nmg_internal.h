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
// (i, j) lives in colour (i + j) & 1 at slot (j, i >> 1) of a [ny][W]
// plane, W = (nx + 1) / 2.  Vectors are [colour][NC][ny][W]; matrices are
// [colour][NE][ny][W] with entry e = (block * NC + row) * NC + col.
struct LevelGeom {
    int nx, ny, W;
    long plane;             // ny * W
};

inline LevelGeom make_geom(int nx, int ny)
{
    LevelGeom g;
    g.nx = nx;
    g.ny = ny;
    g.W = (nx + 1) / 2;
    g.plane = (long)ny * g.W;
    return g;
}

// Read mode of the other colour in a block SGS half sweep.
enum SweepMode {
    MODE_NORMAL = 0,        // other colour as stored
    MODE_ZERO = 1,          // other colour is zero (not materialized)
    MODE_PROLONG = 2,       // stored value + the parent's coarse correction
    MODE_PROLONG_ZERO = 3   // zero + the parent's coarse correction
};

constexpr int kBlock = 256;

inline int nblocks(long n) { return (int)((n + kBlock - 1) / kBlock); }

// ---- launchers (return hipError_t of the launch) ----
hipError_t launch_isolated(const Phys &P, const double *z, const double *U, unsigned char *iso,
                           hipStream_t s);
hipError_t launch_assemble(const Phys &P, const LevelGeom &G, const double *z, const double *U,
                           const unsigned char *iso, double *A, double *b, double *R_out,
                           double *partial, hipStream_t s);
hipError_t launch_residual(const Phys &P, const double *z, const double *U, double *R_out,
                           double *partial, hipStream_t s);
hipError_t launch_reduce(const double *partial, int n, double *out, hipStream_t s);
hipError_t launch_count_u8(const unsigned char *v, long n, double *partial, hipStream_t s);
hipError_t launch_blu_half(const Phys &P, const double *z, double *U, int color, hipStream_t s);
hipError_t launch_update(const Phys &P, const LevelGeom &G, const double *x, double *U,
                         hipStream_t s);
hipError_t launch_threshold(const Phys &P, double *U, hipStream_t s);

hipError_t launch_sgs_half(int dim, int mode, const LevelGeom &G, const double *A, const double *b,
                           double *x, int color, const LevelGeom &Gc, const double *xc,
                           hipStream_t s);
hipError_t launch_restrict(int dim, const LevelGeom &G, const double *A, const double *b,
                           const double *x, const LevelGeom &Gc, double *bc, hipStream_t s);
hipError_t launch_galerkin(int dim, const LevelGeom &Gf, const double *Af, const LevelGeom &Gc,
                           double *Ac, hipStream_t s);
// Materialize one colour of x: op 0 = set zero, 1 = add the parent's
// coarse value, 2 = set to the parent's coarse value.
hipError_t launch_fix_color(int dim, int op, const LevelGeom &G, double *x, int color,
                            const LevelGeom &Gc, const double *xc, hipStream_t s);

// Layout conversions between the public layouts and the colour-split one.
hipError_t launch_vec_to_split(int nc, const LevelGeom &G, const double *v, double *split,
                               hipStream_t s);
hipError_t launch_vec_from_split(int nc, const LevelGeom &G, const double *split, double *v,
                                 hipStream_t s);
hipError_t launch_mat_to_split(int ne, const LevelGeom &G, const double *A, double *split,
                               hipStream_t s);
hipError_t launch_mat_from_split(int ne, const LevelGeom &G, const double *split, double *A,
                                 hipStream_t s);

}  // namespace nmg
