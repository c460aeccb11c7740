// gfx950 kernels of the Newton multigrid method for steady shallow water
// equations (Wu & Tang, arXiv:1608.06721).
//
// All arithmetic is FP64 and must be compiled with -ffp-contract=off: the
// order of every floating-point expression below is fixed (it is part of the
// method's definition in this library), so that results are deterministic
// and independent of launch shapes.
//
// Discretization (Sec. 2.1): hydrostatic reconstruction, HLL or LLF face
// flux evaluated once per face in the +x / +y orientation (exactly
// conservative), edge term F - S(h_own) on the lower-coordinate side and
// -F + S(h_own) on the other, ghost states from the Remark on boundary
// conditions.  Linearization (Sec. 2.2): forward differences with an
// absolute step, alpha ||R_i||_1 on the diagonal.  Multigrid (Sec. 2.3):
// Galerkin sums of child blocks, restriction of the linear residual,
// piecewise-constant prolongation, red-black block Gauss-Seidel.
#include "nmg_sgs.h"

#include <algorithm>

namespace nmg {
namespace {

__device__ __forceinline__ double dmax(double a, double b) { return a > b ? a : b; }
__device__ __forceinline__ double dmin(double a, double b) { return a < b ? a : b; }
__device__ __forceinline__ double dsqrt(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ double dabs(double x) { return __builtin_fabs(x); }
__device__ __forceinline__ bool finite(double x) { return __builtin_isfinite(x); }

// One side of a face: depth, velocity components, bed.
struct Side {
    double h, u, v, z;
};

template <int NC>
struct Cell {
    double q[NC];
};

// ---------------------------------------------------------------------------
// Physical flux along axis 0 (x) or 1 (y): m = h u_n, p = 0.5 g h h,
// (m, m u [+ p], m v [+ p]).
template <int NC>
__device__ __forceinline__ void phys_flux(int axis, double g, double h, double u, double v,
                                          double *F)
{
    double un = (axis == 0) ? u : v;
    double m = h * un;
    double p = 0.5 * g * h * h;
    F[0] = m;
    F[1] = (axis == 0) ? m * u + p : m * u;
    if (NC == 3) F[2] = (axis == 1) ? m * v + p : m * v;
}

// Face flux in the +axis orientation between reconstructed left and right
// states (Remark on numerical fluxes: HLL with two-rarefaction star
// estimates, HLLC, or LLF with the eps_r-enlarged wave speed).
template <int NC>
__device__ __forceinline__ void num_flux(const Phys &P, int axis, double hL, double uL, double vL,
                                         double hR, double uR, double vR, double *out)
{
    const double g = P.g;
    double FL[3], FR[3], UL[3], UR[3];
    phys_flux<NC>(axis, g, hL, uL, vL, FL);
    phys_flux<NC>(axis, g, hR, uR, vR, FR);
    UL[0] = hL; UL[1] = hL * uL; UL[2] = hL * vL;
    UR[0] = hR; UR[1] = hR * uR; UR[2] = hR * vR;
    double unL = (axis == 0) ? uL : vL;
    double unR = (axis == 0) ? uR : vR;
    double cL = dsqrt(g * hL), cR = dsqrt(g * hR);
    if (P.flux == 1) {
        // sqrt(g max(hL, hR)) is max(cL, cR) bit for bit: with g > 0 the
        // rounded product and the correctly rounded square root are monotone
        // and keep the sign of zero, and dmax returns its second operand on
        // ties, so both forms pick the same operand's value.
        double s = dmax(dabs(unL) + cL, dabs(unR) + cR) + P.eps_r * dmax(cL, cR);
#pragma unroll
        for (int k = 0; k < NC; ++k) out[k] = 0.5 * ((FL[k] + FR[k]) - s * (UR[k] - UL[k]));
        return;
    }
    double us = ((unL + unR) * 0.5 + cL) - cR;
    double a = (cL + cR) + (unL - unR) * 0.5;
    double hs = (a * a) / (4.0 * g);
    double cs = dsqrt(g * hs);
    double sL = (hL == 0.0) ? unR - 2.0 * cR : dmin(unL - cL, us - cs);
    double sR = (hR == 0.0) ? unL + 2.0 * cL : dmax(unR + cR, us + cs);
    if (sL >= 0.0) {
#pragma unroll
        for (int k = 0; k < NC; ++k) out[k] = FL[k];
    } else if (sR <= 0.0) {
#pragma unroll
        for (int k = 0; k < NC; ++k) out[k] = FR[k];
    } else {
#pragma unroll
        for (int k = 0; k < NC; ++k)
            out[k] = ((sR * FL[k] - sL * FR[k]) + (sL * sR) * (UR[k] - UL[k])) / (sR - sL);
        if (NC == 3 && P.flux == 2) {
            // HLLC: tangential momentum = upwind tangential velocity (by the
            // sign of the contact speed s_M) times the HLL mass flux; s_M's
            // 0/0 (both sides dry) counts as 0.
            double num = (sL * hR) * (unR - sR) - (sR * hL) * (unL - sL);
            double den = hR * (unR - sR) - hL * (unL - sL);
            double sM = (den != 0.0) ? num / den : 0.0;
            double utL = (axis == 0) ? vL : uL, utR = (axis == 0) ? vR : uR;
            double ut = (sM >= 0.0) ? utL : utR;
            out[2 - axis] = ut * out[0];
        }
    }
}

// Positive root of 2c^3 - K c^2 - gq = 0 by monotone Newton from above.
__device__ double inflow_celerity(double K, double gq)
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

// Ghost cell state behind side f for the interior side `in`.
__device__ Side ghost(const Phys &P, int f, const Side &in)
{
    const SideDev &bc = P.bc[f];
    const double g = P.g;
    int axis = (f == FW || f == FE) ? 0 : 1;
    double sgn = (f == FW || f == FS) ? -1.0 : 1.0;
    double un_in = sgn * (axis == 0 ? in.u : in.v);
    double ut_in = (axis == 0) ? in.v : in.u;
    double hg, ung, utg;
    if (bc.kind == 0) {
        hg = in.h; ung = -un_in; utg = ut_in;
    } else if (bc.kind == 1) {
        hg = in.h; ung = 0.0; utg = ut_in;
    } else {
        bool super = (in.h > P.h_eps) && (in.u * in.u + in.v * in.v >= g * in.h);
        bool outflow = un_in >= 0.0;
        if (super && outflow) {
            hg = in.h; ung = un_in; utg = ut_in;
        } else if (super && bc.hasq && bc.hash && bc.hast) {
            hg = bc.h; ung = -bc.qn / bc.h; utg = bc.ut;
        } else if (bc.hasq && (!bc.hash || !outflow)) {
            double K = un_in + 2.0 * dsqrt(g * in.h);
            double c = inflow_celerity(K, g * bc.qn);
            hg = c * c / g;
            ung = -bc.qn / hg;
            utg = bc.hast ? bc.ut : 0.0;
        } else {
            hg = bc.h;
            ung = (un_in + 2.0 * dsqrt(g * in.h)) - 2.0 * dsqrt(g * hg);
            utg = ut_in;
        }
    }
    Side o;
    o.h = hg;
    o.z = in.z;
    if (axis == 0) { o.u = sgn * ung; o.v = utg; }
    else           { o.u = utg;       o.v = sgn * ung; }
    return o;
}

__device__ __forceinline__ double vel(const Phys &P, double h, double m)
{
    return h > P.h_eps ? m / h : 0.0;
}

template <int NC>
__device__ __forceinline__ Side cell_side(const Phys &P, const double *q, double z)
{
    Side s;
    s.h = q[0];
    s.u = vel(P, q[0], q[1]);
    s.v = (NC == 3) ? vel(P, q[0], q[2]) : 0.0;
    s.z = z;
    return s;
}

// Edge term of eq:totalFlux for the cell on side `own` of face f.
template <int NC>
__device__ __forceinline__ void edge_term(const Phys &P, int f, const Side &own, const Side &oth,
                                          double *T)
{
    int axis = (f == FW || f == FE) ? 0 : 1;
    bool own_left = (f == FE || f == FN);
    const Side &L = own_left ? own : oth;
    const Side &R = own_left ? oth : own;
    double zM = dmax(L.z, R.z);
    double hL = dmax(0.0, L.h + L.z - zM);
    double hR = dmax(0.0, R.h + R.z - zM);
    double F[3];
    num_flux<NC>(P, axis, hL, L.u, L.v, hR, R.u, R.v, F);
    double ho = own_left ? hL : hR;
    double po = 0.5 * P.g * ho * ho;
#pragma unroll
    for (int k = 0; k < NC; ++k) T[k] = own_left ? F[k] : -F[k];
    if (own_left) T[1 + axis] = F[1 + axis] - po;
    else          T[1 + axis] = -F[1 + axis] + po;
}

__device__ __forceinline__ bool neighbour(const Phys &P, int i, int j, int f, int &ni, int &nj)
{
    ni = i;
    nj = j;
    if (f == FW) { ni = i - 1; return i > 0; }
    if (f == FE) { ni = i + 1; return i + 1 < P.nx; }
    if (f == FS) { nj = j - 1; return j > 0; }
    nj = j + 1;
    return j + 1 < P.ny;
}

template <int NC>
__device__ __forceinline__ void load_state(const Phys &P, const double *U, long idx, double *q)
{
    const long N = (long)P.nx * P.ny;
#pragma unroll
    for (int k = 0; k < NC; ++k) q[k] = U[k * N + idx];
}

// Deterministic block reduction of one double per thread; thread 0 of the
// block receives the sum.  Fixed pairing order, so the result depends only
// on the block size, never on timing.
__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double sh[kBlock];
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
#pragma unroll
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] = sh[t] + sh[t + s];
        __syncthreads();
    }
    return sh[0];
}

// Value of lane Q of each aligned group of four lanes, in all four (DPP
// quad_perm broadcast).
template <int Q>
__device__ __forceinline__ double quad_bcast(double v)
{
    constexpr int kCtrl = Q * 0x55;     // quad_perm [Q, Q, Q, Q]
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)u, kCtrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), kCtrl, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Residual and forward-difference blocks of one cell.  D receives
// sum_e |e| dT/dU_i, Off[f] receives |e| dT/dU_j for interior faces.
// Off-diagonal blocks are handed to `off(f, r, k, value)` as soon as face f
// is done (value 0 on boundary faces), so no per-face array is kept.  The
// face loop is unrolled, so that each face's orientation (which side is
// left, which momentum is normal) is fixed at compile time instead of being
// selected per evaluation: about 30 % fewer instructions.
struct NoOff {
    __device__ void operator()(int, int, int, double) const {}
};

// The states and beds of a cell's face neighbours, loaded together so that
// their latencies overlap (a boundary face holds the cell itself, unused).
template <int NC>
struct Nbrs {
    double q[4][NC], z[4];
    bool inner[4];
};

// An empty register constraint on the neighbours' values: the compiler must
// take them as changed here, so arithmetic on them stays inside a loop of
// cell updates instead of being hoisted out of it and kept live in extra
// registers across the loop.
template <int NC>
__device__ __forceinline__ void opaque_nbrs(Nbrs<NC> &nb)
{
    const int NF = (NC == 2) ? 2 : 4;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int c = 0; c < NC; ++c) asm volatile("" : "+v"(nb.q[f][c]));
        asm volatile("" : "+v"(nb.z[f]));
    }
}

template <int NC>
__device__ __forceinline__ void load_nbrs(const Phys &P, const double *z, const double *U, int i,
                                          int j, Nbrs<NC> &nb)
{
    const int NF = (NC == 2) ? 2 : 4;
    const long idx = (long)j * P.nx + i;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        int ni, nj;
        nb.inner[f] = neighbour(P, i, j, f, ni, nj);
        const long nidx = nb.inner[f] ? (long)nj * P.nx + ni : idx;
        load_state<NC>(P, U, nidx, nb.q[f]);
        nb.z[f] = z[nidx];
    }
}

// cell_jacobian at the cell state qi (bed zi).  With PRE the neighbours come
// from nb; otherwise each face loads its own (with the off-diagonal blocks,
// loading them all first would take the kernel past 256 registers).
template <int NC, bool WANT_OFF, bool PRE, class OffSink>
__device__ __forceinline__ void cell_jacobian_at(const Phys &P, const double *z, const double *U,
                                                 int i, int j, const double *qi, double zi,
                                                 const Nbrs<NC> &nb, double *Rc, double (*D)[NC],
                                                 const OffSink &off)
{
    const int NF = (NC == 2) ? 2 : 4;
    const double eps = P.eps;
    Side own = cell_side<NC>(P, qi, zi);
    Side ownp[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        double qp[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) qp[c] = qi[c];
        qp[k] = qp[k] + eps;
        ownp[k] = cell_side<NC>(P, qp, zi);
    }
#pragma unroll
    for (int r = 0; r < NC; ++r) {
        Rc[r] = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) D[r][c] = 0.0;
    }
    auto face = [&](int f) {
        const double e = P.elen[f];
        double T0[NC], Tk[NC];
        bool inner;
        double qj[NC], zj;
        if constexpr (PRE) {
            inner = nb.inner[f];
#pragma unroll
            for (int c = 0; c < NC; ++c) qj[c] = nb.q[f][c];
            zj = nb.z[f];
        } else {
            int ni, nj;
            inner = neighbour(P, i, j, f, ni, nj);
            if (inner) {
                const long nidx = (long)nj * P.nx + ni;
                load_state<NC>(P, U, nidx, qj);
                zj = z[nidx];
            }
        }
        if (inner) {
            Side oth = cell_side<NC>(P, qj, zj);
            edge_term<NC>(P, f, own, oth, T0);
#pragma unroll
            for (int r = 0; r < NC; ++r) Rc[r] = Rc[r] + e * T0[r];
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                edge_term<NC>(P, f, ownp[k], oth, Tk);
#pragma unroll
                for (int r = 0; r < NC; ++r) D[r][k] = D[r][k] + e * ((Tk[r] - T0[r]) / eps);
            }
            if (WANT_OFF) {
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    double qp[NC];
#pragma unroll
                    for (int c = 0; c < NC; ++c) qp[c] = qj[c];
                    qp[k] = qp[k] + eps;
                    Side othp = cell_side<NC>(P, qp, zj);
                    edge_term<NC>(P, f, own, othp, Tk);
#pragma unroll
                    for (int r = 0; r < NC; ++r) off(f, r, k, e * ((Tk[r] - T0[r]) / eps));
                }
            }
        } else {
            Side gh = ghost(P, f, own);
            edge_term<NC>(P, f, own, gh, T0);
#pragma unroll
            for (int r = 0; r < NC; ++r) Rc[r] = Rc[r] + e * T0[r];
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                Side ghp = ghost(P, f, ownp[k]);
                edge_term<NC>(P, f, ownp[k], ghp, Tk);
#pragma unroll
                for (int r = 0; r < NC; ++r) D[r][k] = D[r][k] + e * ((Tk[r] - T0[r]) / eps);
            }
            if (WANT_OFF) {
#pragma unroll
                for (int r = 0; r < NC; ++r)
#pragma unroll
                    for (int c = 0; c < NC; ++c) off(f, r, c, 0.0);
            }
        }
    };
#pragma unroll
    for (int f = 0; f < NF; ++f) face(f);
}

template <int NC, bool WANT_OFF, class OffSink>
__device__ __forceinline__ void cell_jacobian(const Phys &P, const double *z, const double *U, int i,
                                              int j, double *Rc, double (*D)[NC], const OffSink &off)
{
    const long idx = (long)j * P.nx + i;
    double qi[NC];
    load_state<NC>(P, U, idx, qi);
    Nbrs<NC> none;
    cell_jacobian_at<NC, WANT_OFF, false>(P, z, U, i, j, qi, z[idx], none, Rc, D, off);
}

template <int NC>
__device__ __forceinline__ double l1norm(const double *Rc)
{
    double s = dabs(Rc[0]) + dabs(Rc[1]);
    if (NC == 3) s = s + dabs(Rc[2]);
    return s;
}

// ---------------------------------------------------------------------------
// Kernels on the natural (public) layout.

// Isolation flag of cell idx: zero reconstructed depth on both sides of
// every face.
template <int NC>
__device__ __forceinline__ void isolated_cell(const Phys &P, const double *__restrict__ z,
                                              const double *__restrict__ U,
                                              unsigned char *__restrict__ iso, long idx)
{
    const int NF = (NC == 2) ? 2 : 4;
    int i = (int)(idx % P.nx), j = (int)(idx / P.nx);
    double qi[NC];
    load_state<NC>(P, U, idx, qi);
    Side own = cell_side<NC>(P, qi, z[idx]);
    unsigned char res = 1;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        int ni, nj;
        Side oth;
        if (neighbour(P, i, j, f, ni, nj)) {
            long nidx = (long)nj * P.nx + ni;
            double qj[NC];
            load_state<NC>(P, U, nidx, qj);
            oth = cell_side<NC>(P, qj, z[nidx]);
        } else {
            oth = ghost(P, f, own);
        }
        double zM = dmax(own.z, oth.z);
        double h1 = dmax(0.0, own.h + own.z - zM);
        double h2 = dmax(0.0, oth.h + oth.z - zM);
        if (h1 != 0.0 || h2 != 0.0) res = 0;
    }
    iso[idx] = res;
}

template <int NC>
__global__ void __launch_bounds__(kBlock) k_isolated(Phys P, const double *__restrict__ z,
                                                     const double *__restrict__ U,
                                                     unsigned char *__restrict__ iso)
{
    long idx = (long)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (long)P.nx * P.ny) return;
    isolated_cell<NC>(P, z, U, iso, idx);
}

// Stores the off-diagonal blocks of one cell in the colour-split layout,
// applying the pinning rules: an isolated cell gets a zero row, a dry cell
// under the dry-cell pin zero momentum rows, and the column of an isolated
// neighbour is zero.
template <int NC, class T>
struct OffStore {
    T *Ac;                 // this cell's entry 0 in the colour-split matrix
    bool me_iso, dryp;
    bool nb_iso[4];
    __device__ void operator()(int f, int r, int c, double v) const
    {
        if (me_iso || nb_iso[f] || (dryp && r > 0)) v = 0.0;
        Ac[(((f + 1) * NC + r) * NC + c) * kTile] = T(v);
    }
};

// Residual, Jacobian blocks and right-hand side of cell idx; returns
// ||R_i||_1.  The blocks and b are computed in FP64 and stored in the
// hierarchy's precision T (rounded to nearest when T is float).
template <int NC, class T>
__device__ __forceinline__ double assemble_cell(const Phys &P, const LevelGeom &G,
                                                const double *__restrict__ z,
                                                const double *__restrict__ U,
                                                const unsigned char *__restrict__ iso,
                                                T *__restrict__ A, T *__restrict__ b,
                                                double *__restrict__ R_out, long idx)
{
    const int NF = (NC == 2) ? 2 : 4;
    const int NE = (NF + 1) * NC * NC;
    const long N = (long)P.nx * P.ny;
    double nrm = 0.0;
    {
        int i = (int)(idx % P.nx), j = (int)(idx / P.nx);
        const int color = (i + j) & 1;
        const long slot = (long)j * G.W + (i >> 1);
        OffStore<NC, T> st;
        st.Ac = A + mat_off(G, NE, color, slot);
        st.me_iso = iso[idx] != 0;
        st.dryp = !st.me_iso && P.dry_pin && U[idx] == 0.0;
        for (int f = 0; f < 4; ++f) {
            int ni, nj;
            st.nb_iso[f] = f < NF && neighbour(P, i, j, f, ni, nj) && iso[(long)nj * P.nx + ni];
        }
        double Rc[NC], D[NC][NC];
        cell_jacobian<NC, true>(P, z, U, i, j, Rc, D, st);
        if (R_out) {
#pragma unroll
            for (int r = 0; r < NC; ++r) R_out[r * N + idx] = Rc[r];
        }
        nrm = l1norm<NC>(Rc);
#pragma unroll
        for (int r = 0; r < NC; ++r) D[r][r] = D[r][r] + P.alpha * nrm;
        if (st.me_iso) {
#pragma unroll
            for (int r = 0; r < NC; ++r)
#pragma unroll
                for (int c = 0; c < NC; ++c) D[r][c] = 0.0;
        } else if (st.dryp) {
#pragma unroll
            for (int r = 1; r < NC; ++r) {
#pragma unroll
                for (int c = 0; c < NC; ++c) D[r][c] = 0.0;
                D[r][r] = D[0][0];
                Rc[r] = 0.0;
            }
        }
        T *bc = b + (long)color * NC * G.plane + slot;
#pragma unroll
        for (int r = 0; r < NC; ++r) {
            bc[r * G.plane] = T(st.me_iso ? 0.0 : -Rc[r]);
#pragma unroll
            for (int c = 0; c < NC; ++c) st.Ac[(r * NC + c) * kTile] = T(D[r][c]);
        }
    }
    return nrm;
}

template <int NC, class T>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) k_assemble(Phys P, LevelGeom G,
                                                     const double *__restrict__ z,
                                                     const double *__restrict__ U,
                                                     const unsigned char *__restrict__ iso,
                                                     T *__restrict__ A,
                                                     T *__restrict__ b,
                                                     double *__restrict__ R_out,
                                                     double *__restrict__ partial)
{
    const int xb = xcd_block(blockIdx.x, gridDim.x);
    long idx = (long)xb * kBlock + threadIdx.x;
    double nrm = 0.0;
    if (idx < (long)P.nx * P.ny) nrm = assemble_cell<NC, T>(P, G, z, U, iso, A, b, R_out, idx);
    double s = block_sum(nrm);
    if (threadIdx.x == 0) partial[xb] = s;
}

// Residual R_i (eq:Res) of cell idx, optionally stored; returns ||R_i||_1.
template <int NC>
__device__ __forceinline__ double residual_cell(const Phys &P, const double *__restrict__ z,
                                                const double *__restrict__ U,
                                                double *__restrict__ R_out, long idx)
{
    const int NF = (NC == 2) ? 2 : 4;
    const long N = (long)P.nx * P.ny;
    double nrm = 0.0;
    {
        int i = (int)(idx % P.nx), j = (int)(idx / P.nx);
        double qi[NC];
        load_state<NC>(P, U, idx, qi);
        Side own = cell_side<NC>(P, qi, z[idx]);
        double Rc[NC];
#pragma unroll
        for (int r = 0; r < NC; ++r) Rc[r] = 0.0;
        Nbrs<NC> nb;
        load_nbrs<NC>(P, z, U, i, j, nb);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            Side oth;
            if (nb.inner[f]) {
                oth = cell_side<NC>(P, nb.q[f], nb.z[f]);
            } else {
                oth = ghost(P, f, own);
            }
            double T[NC];
            edge_term<NC>(P, f, own, oth, T);
#pragma unroll
            for (int r = 0; r < NC; ++r) Rc[r] = Rc[r] + P.elen[f] * T[r];
        }
        if (R_out) {
#pragma unroll
            for (int r = 0; r < NC; ++r) R_out[r * N + idx] = Rc[r];
        }
        nrm = l1norm<NC>(Rc);
    }
    return nrm;
}

template <int NC>
__global__ void __launch_bounds__(kBlock) k_residual(Phys P, const double *__restrict__ z,
                                                     const double *__restrict__ U,
                                                     double *__restrict__ R_out,
                                                     double *__restrict__ partial)
{
    const int xb = xcd_block(blockIdx.x, gridDim.x);
    long idx = (long)xb * kBlock + threadIdx.x;
    double nrm = 0.0;
    if (idx < (long)P.nx * P.ny) nrm = residual_cell<NC>(P, z, U, R_out, idx);
    double s = block_sum(nrm);
    if (threadIdx.x == 0) partial[xb] = s;
}

// Sum of n block partials in a fixed order (one block): thread t sums
// partials t, t + kBlock, ..., then the block's tree; thread 0 holds the sum.
__device__ __forceinline__ double sum_partials(const double *__restrict__ partial, int n)
{
    double v = 0.0;
    for (int k = threadIdx.x; k < n; k += kBlock) v = v + partial[k];
    return block_sum(v);
}

__global__ void __launch_bounds__(kBlock) k_reduce(const double *__restrict__ partial, int n,
                                                   double *__restrict__ out)
{
    double s = sum_partials(partial, n);
    if (threadIdx.x == 0) out[0] = s;
}

__global__ void k_step1_reset(int *__restrict__ ctrl)
{
    ctrl[0] = 0;
    ctrl[1] = 0;
    ctrl[2] = 0;
    ctrl[3] = 0;
}

__global__ void __launch_bounds__(kBlock) k_count_u8(const unsigned char *__restrict__ v, long n,
                                                     double *__restrict__ partial)
{
    long idx = (long)blockIdx.x * kBlock + threadIdx.x;
    double c = (idx < n && v[idx]) ? 1.0 : 0.0;
    double s = block_sum(c);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// The regularized block of one BLU-SGS update and its solution: D gets
// alpha ||R_i||_1 on its diagonal, a dry cell under the dry-cell pin (h = 0)
// keeps only its depth row, and d solves D d = R_i; then the new state
// q - d, with the dry threshold (every component 0 below h_eps).
template <int NC>
__device__ __forceinline__ double blu_solve(const Phys &P, double *Rc, double (*D)[NC], double *q)
{
    const double nrm = l1norm<NC>(Rc);
#pragma unroll
    for (int r = 0; r < NC; ++r) D[r][r] = D[r][r] + P.alpha * nrm;
    if (P.dry_pin && q[0] == 0.0) {
#pragma unroll
        for (int r = 1; r < NC; ++r) {
#pragma unroll
            for (int c = 0; c < NC; ++c) D[r][c] = 0.0;
            D[r][r] = D[0][0];
            Rc[r] = 0.0;
        }
    }
    double M[NC * NC], d[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c) M[r * NC + c] = D[r][c];
    solve_block<double, NC>(M, Rc, d);
#pragma unroll
    for (int c = 0; c < NC; ++c) q[c] = q[c] - d[c];
    if (q[0] < P.h_eps) {
#pragma unroll
        for (int c = 0; c < NC; ++c) q[c] = 0.0;
    }
    return nrm;
}

// Edge term |e_f| T_f of face f of the cell in slot t of `color`, at state
// U, as residual_cell forms it; false if the slot holds no cell.
template <int NC>
__device__ __forceinline__ bool slot_face_term(const Phys &P, const double *__restrict__ z,
                                               const double *__restrict__ U, int color, long t,
                                               int f, double *eT)
{
    const int W = (P.nx + 1) / 2;
    int j = (int)(t / W), k = (int)(t % W);
    int i = 2 * k + ((j + color) & 1);
    if (i >= P.nx) return false;
    const long idx = (long)j * P.nx + i;
    double qi[NC];
    load_state<NC>(P, U, idx, qi);
    const Side own = cell_side<NC>(P, qi, z[idx]);
    int ni, nj;
    Side oth;
    if (neighbour(P, i, j, f, ni, nj)) {
        const long nidx = (long)nj * P.nx + ni;
        double qj[NC];
        load_state<NC>(P, U, nidx, qj);
        oth = cell_side<NC>(P, qj, z[nidx]);
    } else {
        oth = ghost(P, f, own);
    }
    double T[NC];
    edge_term<NC>(P, f, own, oth, T);
#pragma unroll
    for (int r = 0; r < NC; ++r) eT[r] = P.elen[f] * T[r];
    return true;
}

// ||R_i||_1 of the cell in slot t of `color` at state U (0 if none).
template <int NC>
__device__ __forceinline__ double slot_residual_norm(const Phys &P, const double *__restrict__ z,
                                                     const double *__restrict__ U, int color,
                                                     long t)
{
    const int W = (P.nx + 1) / 2;
    int j = (int)(t / W), k = (int)(t % W);
    int i = 2 * k + ((j + color) & 1);
    if (i >= P.nx) return 0.0;
    return residual_cell<NC>(P, z, U, nullptr, (long)j * P.nx + i);
}

// One BLU-SGS cell update for every cell of one colour (Algorithm 1,
// Step 2.1): U_i -= (alpha ||R_i||_1 I + dR_i/dU_i)^-1 R_i, then the dry
// threshold.  Cells of one colour only read the other colour, so `reps`
// consecutive half sweeps of the same colour are `reps` updates of each cell
// from its neighbours' unchanged states: one launch does them with the
// state kept in registers, the same arithmetic as `reps` launches.
// blu_cell_update reads the cell's own state from Uown and its neighbours'
// from Unb (the other colour), leaves the new state in q, the cell's index
// in idx and ||R_i||_1 at the starting state in nrm0; false if slot t of the
// colour holds no cell.
template <int NC>
__device__ __forceinline__ bool blu_cell_update(const Phys &P, const double *__restrict__ z,
                                                const double *Uown, const double *Unb,
                                                int color, long t, int reps, double *q, long &idx,
                                                double &nrm0)
{
    const int W = (P.nx + 1) / 2;
    int j = (int)(t / W), k = (int)(t % W);
    int i = 2 * k + ((j + color) & 1);
    if (i >= P.nx) return false;
    idx = (long)j * P.nx + i;
    load_state<NC>(P, Uown, idx, q);
    const double zi = z[idx];
    Nbrs<NC> nb;
    load_nbrs<NC>(P, z, Unb, i, j, nb);
    for (int rep = 0; rep < reps; ++rep) {
        opaque_nbrs<NC>(nb);
        double Rc[NC], D[NC][NC];
        cell_jacobian_at<NC, false, true>(P, z, Unb, i, j, q, zi, nb, Rc, D, NoOff());
        const double nrm = blu_solve<NC>(P, Rc, D, q);
        if (rep == 0) nrm0 = nrm;
    }
    return true;
}

template <int NC>
__device__ __forceinline__ void blu_cell(const Phys &P, const double *__restrict__ z,
                                         double *__restrict__ U, int color, long t)
{
    const long N = (long)P.nx * P.ny;
    double q[NC], nrm0;
    long idx;
    if (!blu_cell_update<NC>(P, z, U, U, color, t, 1, q, idx, nrm0)) return;
#pragma unroll
    for (int c = 0; c < NC; ++c) U[c * N + idx] = q[c];
}

// Sum of one double per thread over the block for the Step 1 stop test:
// each wave's lane 0 sums its wave by a butterfly of lane exchanges, then
// every thread adds the waves' sums in wave order, so all threads hold the
// same value.  Two barriers instead of block_sum's eight (the order of this
// sum is the GPU's own: the oracle sums the cells in index order, and only
// the comparison with the threshold uses it).
__device__ __forceinline__ double block_sum_step1(double v)
{
    constexpr int kWaves = kBlock / 64;
    __shared__ double ws[kWaves];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = v + __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s = s + ws[w];
    __syncthreads();
    return s;
}

// This thread's share of the stop test's partials (the first stage of
// sum_partials), loaded before the cell's arithmetic so their latency
// overlaps it.
__device__ __forceinline__ double stop_share(const StopTest &st)
{
    double v = 0.0;
    if (st.partial)
        for (int k = threadIdx.x; k < st.n; k += kBlock) v = v + st.partial[k];
    return v;
}

// The Step 1 stop flag: block 0 of the launch that takes the decision sets it
// while other blocks of that launch may read it, so it is accessed with
// relaxed atomics (a set flag only ever agrees with their own decision).
__device__ __forceinline__ bool flag_set(const int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// The stop decision of a launch with a stop test; every thread of the block
// takes part (block_sum_step1 synchronizes) and gets the same answer.
__device__ __forceinline__ bool stop_decision(const StopTest &st, double share)
{
    if (!st.partial) return false;
    const bool stopped = flag_set(st.ctrl);
    const int done = st.ctrl[2 + st.parity];
    const double s = block_sum_step1(share);
    const bool stop = stopped || !(s >= st.thr) || done >= st.max_sweeps;
    if (!stopped && blockIdx.x == 0 && threadIdx.x == 0) {
        if (stop) {
            st.ctrl[1] = done;
            __hip_atomic_store(st.ctrl, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            st.ctrl[2 + (st.parity ^ 1)] = done + 1;
        }
    }
    return stop;
}

// Block partial of a launch's residual output (res_partial[xb]): the sum of
// its threads' norms.
__device__ __forceinline__ void residual_partial(double *res_partial, int xb, double nrm)
{
    const double s = block_sum_step1(nrm);
    if (threadIdx.x == 0) res_partial[xb] = s;
}

// A BLU-SGS half sweep: the cells of `color` read their own state from Uown
// and their neighbours' from Unb, and store the new state to Uout (all
// three the same array for an in-place half sweep).  gate (nullable): a
// flag set by the Step 1 stop test of an earlier launch; once it is set the
// launch stores nothing.  It is read with the cell's data and tested only
// before the store, so its latency overlaps the arithmetic; so is this
// launch's own stop test (st).  res_partial (nullable, Uown == Unb): the
// launch also writes, per block, the sum of ||R_i||_1 at the input state of
// its slots' cells of both colours (the next launch's stop test reads them).
template <int NC>
__global__ void __launch_bounds__(kBlock) k_blu_half(Phys P, const double *__restrict__ z,
                                                     const double *Uown, const double *Unb,
                                                     double *Uout, int color, int reps,
                                                     const int *__restrict__ gate, StopTest st,
                                                     double *__restrict__ res_partial)
{
    const int W = (P.nx + 1) / 2;
    const int xb = xcd_block(blockIdx.x, gridDim.x);
    const long t = (long)xb * kBlock + threadIdx.x;
    const long N = (long)P.nx * P.ny;
    const bool slot = t < (long)W * P.ny;
    const double share = stop_share(st);
    double q[NC], nrm = 0.0;
    long idx = 0;
    const bool cell = slot && blu_cell_update<NC>(P, z, Uown, Unb, color, t, reps, q, idx, nrm);
    if (res_partial) {
        if (!cell) nrm = 0.0;
        if (slot) nrm = nrm + slot_residual_norm<NC>(P, z, Uown, color ^ 1, t);
        residual_partial(res_partial, xb, nrm);
    }
    const bool stop = stop_decision(st, share);
    if (!cell || stop || (gate && flag_set(gate))) return;
#pragma unroll
    for (int c = 0; c < NC; ++c) Uout[c * N + idx] = q[c];
}

// blu_cell with four lanes per cell, lane k of the cell's aligned quad
// (the lanes of a cell run in lockstep in one wave).  Lane 0 evaluates each
// face's edge term at the cell's state, lane k = 1..NC the edge term with
// component k-1 of the cell's state perturbed (ghost states re-evaluated from
// that perturbed state on boundary faces); per face the unperturbed term is
// broadcast from lane 0 and lane k accumulates column k-1 of the diagonal
// block, lane 0 the residual, each in the face order W, E, S, N.  After the
// faces every lane gathers R_i and the block, and does the regularization,
// the pin, the block solve and the threshold; lane 0 stores.  Each sum,
// difference quotient and product is blu_cell's, in its order, so the result
// is the same bit for bit; a cell's longest chain of dependent arithmetic is
// one edge term (and ghost) per face instead of NC + 1.
template <int NC>
__device__ __forceinline__ bool blu_cell_quad(const Phys &P, const double *__restrict__ z,
                                              const double *Uown, const double *Unb, int color,
                                              long t, int k, int reps, double *qi, long &idx,
                                              double &nrm0)
{
    const int NF = (NC == 2) ? 2 : 4;
    const int W = (P.nx + 1) / 2;
    int j = (int)(t / W), kk = (int)(t % W);
    int i = 2 * kk + ((j + color) & 1);
    if (i >= P.nx) return false;
    idx = (long)j * P.nx + i;
    const double eps = P.eps;
    load_state<NC>(P, Uown, idx, qi);
    const double zi = z[idx];
    Nbrs<NC> nb;
    load_nbrs<NC>(P, z, Unb, i, j, nb);
    for (int rep = 0; rep < reps; ++rep) {
        opaque_nbrs<NC>(nb);
        // this lane's own side: unperturbed (k = 0) or component k-1 + eps
        double qk[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) qk[c] = qi[c];
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (k == c + 1) qk[c] = qk[c] + eps;
        const Side mine = cell_side<NC>(P, qk, zi);
        double acc[NC];     // lane 0: R_i; lane k: column k-1 of sum_e |e| dT/dU_i
#pragma unroll
        for (int r = 0; r < NC; ++r) acc[r] = 0.0;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const double e = P.elen[f];
            double T[NC], T0[NC];
            if (nb.inner[f]) {
                Side oth = cell_side<NC>(P, nb.q[f], nb.z[f]);
                edge_term<NC>(P, f, mine, oth, T);
            } else {
                Side gh = ghost(P, f, mine);
                edge_term<NC>(P, f, mine, gh, T);
            }
#pragma unroll
            for (int r = 0; r < NC; ++r) T0[r] = quad_bcast<0>(T[r]);
            if (k == 0) {
#pragma unroll
                for (int r = 0; r < NC; ++r) acc[r] = acc[r] + e * T[r];
            } else {
#pragma unroll
                for (int r = 0; r < NC; ++r) acc[r] = acc[r] + e * ((T[r] - T0[r]) / eps);
            }
        }
        double Rc[NC], D[NC][NC];
#pragma unroll
        for (int r = 0; r < NC; ++r) {
            Rc[r] = quad_bcast<0>(acc[r]);
            D[r][0] = quad_bcast<1>(acc[r]);
            D[r][1] = quad_bcast<2>(acc[r]);
            if (NC == 3) D[r][NC - 1] = quad_bcast<3>(acc[r]);
        }
        const double nrm = blu_solve<NC>(P, Rc, D, qi);
        if (rep == 0) nrm0 = nrm;
    }
    return true;
}

// ||R_i||_1 of the cell in slot t of `color` at U with four lanes per cell:
// lane k forms face k's term, lane 0 gets the sum over the faces in the
// order W, E, S, N (residual_cell's), the other lanes 0.  Every lane of the
// quad must take part.
template <int NC>
__device__ __forceinline__ double slot_residual_norm_quad(const Phys &P,
                                                          const double *__restrict__ z,
                                                          const double *__restrict__ U,
                                                          int color, long t, int k)
{
    const int NF = (NC == 2) ? 2 : 4;
    double eT[NC];
    // (in 1D lanes 2 and 3 repeat face 0 and contribute nothing)
    const bool cell = slot_face_term<NC>(P, z, U, color, t, k < NF ? k : 0, eT);
    if (!cell || k >= NF) {
#pragma unroll
        for (int r = 0; r < NC; ++r) eT[r] = 0.0;
    }
    double R[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r) {
        double v = 0.0;
        v = v + quad_bcast<0>(eT[r]);
        v = v + quad_bcast<1>(eT[r]);
        if (NC == 3) {
            v = v + quad_bcast<2>(eT[r]);
            v = v + quad_bcast<3>(eT[r]);
        }
        R[r] = v;
    }
    return (cell && k == 0) ? l1norm<NC>(R) : 0.0;
}

// k_blu_half with four lanes per cell (the arguments are k_blu_half's).
template <int NC>
__global__ void __launch_bounds__(kBlock) k_blu_half_quad(Phys P, const double *__restrict__ z,
                                                          const double *Uown, const double *Unb,
                                                          double *Uout, int color, int reps,
                                                          const int *__restrict__ gate,
                                                          StopTest st,
                                                          double *__restrict__ res_partial)
{
    const int W = (P.nx + 1) / 2;
    const int xb = xcd_block(blockIdx.x, gridDim.x);
    const long g = (long)xb * kBlock + threadIdx.x;
    const long t = g >> 2;
    const int k = (int)(g & 3);
    const long N = (long)P.nx * P.ny;
    // the four lanes of a cell share t, so whole quads are active or not
    const bool slot = t < (long)W * P.ny;
    const double share = stop_share(st);
    // the other colour's residual norm first (lane 0; 0 without output)
    const double nrm1 = (res_partial && slot)
                            ? slot_residual_norm_quad<NC>(P, z, Uown, color ^ 1, t, k) : 0.0;
    double q[NC], nrm = 0.0;
    long idx = 0;
    const bool cell =
        slot && blu_cell_quad<NC>(P, z, Uown, Unb, color, t, k, reps, q, idx, nrm);
    if (res_partial) {
        if (!cell || k != 0) nrm = 0.0;
        residual_partial(res_partial, xb, nrm + nrm1);
    }
    const bool stop = stop_decision(st, share);
    if (!cell || k != 0 || stop || (gate && flag_set(gate))) return;
#pragma unroll
    for (int c = 0; c < NC; ++c) Uout[c * N + idx] = q[c];
}

// Value of lane i + S of the 16-lane row (DPP row_shl:S; lanes whose source
// is past the row's end read garbage that nothing uses).
template <int S>
__device__ __forceinline__ double row_shl(double v)
{
    constexpr int kCtrl = 0x100 + S;
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)u, kCtrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), kCtrl, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Sum over the four faces, in the order W, E, S, N, of the value that lane
// Q of each face's quad holds; valid in lane 0 of the cell's 16 lanes.
template <int Q>
__device__ __forceinline__ double faces_sum(double v)
{
    const double w = quad_bcast<Q>(v);
    double s = 0.0;
    s = s + w;
    s = s + row_shl<4>(w);
    s = s + row_shl<8>(w);
    s = s + row_shl<12>(w);
    return s;
}

// blu_cell for 2D cells with sixteen lanes per cell, one per (face f,
// evaluation k): lane 4 f + k evaluates face f's edge term at the cell's
// state (k = 0) or with component k-1 perturbed (ghost states re-evaluated
// from that state on boundary faces), forms its term of R_i (k = 0) or of
// column k-1 of the diagonal block, |e| ((T_k - T_0) / eps), with T_0 taken
// from lane 4 f; lane 0 of the cell then sums the four faces' terms in the
// order W, E, S, N, and does the regularization, the pin, the block solve,
// the threshold and the store (with reps > 1 it hands the new state to the
// cell's other lanes for the next update).  Every operation is blu_cell's in
// its order, so the result is the same bit for bit; a cell's chain of
// dependent arithmetic is one edge term and one ghost state per update.
__device__ __forceinline__ bool blu_cell_x16(const Phys &P, const double *__restrict__ z,
                                             const double *Uown, const double *Unb, int color,
                                             long t, int lane, int reps, double *qi, long &idx,
                                             double &nrm0)
{
    constexpr int NC = 3;
    const int W = (P.nx + 1) / 2;
    int j = (int)(t / W), kk = (int)(t % W);
    int i = 2 * kk + ((j + color) & 1);
    if (i >= P.nx) return false;
    const int f = lane >> 2, k = lane & 3;
    idx = (long)j * P.nx + i;
    const double eps = P.eps;
    load_state<NC>(P, Uown, idx, qi);
    const double zi = z[idx];
    const double e = P.elen[f];
    int ni, nj;
    const bool inner = neighbour(P, i, j, f, ni, nj);
    const long nidx = inner ? (long)nj * P.nx + ni : idx;
    double qj[NC];
    load_state<NC>(P, inner ? Unb : Uown, nidx, qj);
    const double zj = z[nidx];
    for (int rep = 0; rep < reps; ++rep) {
        if (rep > 0) {
#pragma unroll
            for (int c = 0; c < NC; ++c) qi[c] = __shfl(qi[c], 0, 16);
        }
        double qk[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) qk[c] = qi[c];
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (k == c + 1) qk[c] = qk[c] + eps;
        const Side mine = cell_side<NC>(P, qk, zi);
        double T[NC];
        if (inner) {
            Side oth = cell_side<NC>(P, qj, zj);
            edge_term<NC>(P, f, mine, oth, T);
        } else {
            Side gh = ghost(P, f, mine);
            edge_term<NC>(P, f, mine, gh, T);
        }
        double term[NC];    // lane k = 0: |e| T_0; lane k > 0: |e| (T_k - T_0) / eps
#pragma unroll
        for (int r = 0; r < NC; ++r) {
            const double T0 = quad_bcast<0>(T[r]);
            term[r] = (k == 0) ? e * T[r] : e * ((T[r] - T0) / eps);
        }
        double Rc[NC], D[NC][NC];
#pragma unroll
        for (int r = 0; r < NC; ++r) {
            Rc[r] = faces_sum<0>(term[r]);
            D[r][0] = faces_sum<1>(term[r]);
            D[r][1] = faces_sum<2>(term[r]);
            D[r][2] = faces_sum<3>(term[r]);
        }
        // valid in lane 0 only; the other lanes' results are replaced above
        const double nrm = blu_solve<NC>(P, Rc, D, qi);
        if (rep == 0) nrm0 = nrm;
    }
    return true;
}

// ||R_i||_1 of the cell in slot t of `color` at U with sixteen lanes per
// cell: lane 4 f forms face f's term, lane 0 gets the sum over the faces in
// the order W, E, S, N (residual_cell's), the other lanes 0.  Every lane of
// the row must take part.
__device__ __forceinline__ double slot_residual_norm_x16(const Phys &P,
                                                         const double *__restrict__ z,
                                                         const double *__restrict__ U, int color,
                                                         long t, int lane)
{
    constexpr int NC = 3;
    double eT[NC] = {0.0, 0.0, 0.0};
    bool cell = true;
    if ((lane & 3) == 0) cell = slot_face_term<NC>(P, z, U, color, t, lane >> 2, eT);
    double R[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r) R[r] = faces_sum<0>(eT[r]);
    return (cell && lane == 0) ? l1norm<NC>(R) : 0.0;
}

// k_blu_half with sixteen lanes per cell (2D; the arguments are k_blu_half's).
__global__ void __launch_bounds__(kBlock) k_blu_half_x16(Phys P, const double *__restrict__ z,
                                                         const double *Uown, const double *Unb,
                                                         double *Uout, int color, int reps,
                                                         const int *__restrict__ gate,
                                                         StopTest st,
                                                         double *__restrict__ res_partial)
{
    const int W = (P.nx + 1) / 2;
    const int xb = xcd_block(blockIdx.x, gridDim.x);
    const long g = (long)xb * kBlock + threadIdx.x;
    const long t = g >> 4;
    const int lane = (int)(g & 15);
    const long N = (long)P.nx * P.ny;
    // the sixteen lanes of a cell share t, so whole rows are active or not
    const bool slot = t < (long)W * P.ny;
    const double share = stop_share(st);
    double q[3], nrm = 0.0;
    long idx = 0;
    const bool cell = slot && blu_cell_x16(P, z, Uown, Unb, color, t, lane, reps, q, idx, nrm);
    if (res_partial) {
        if (!cell || lane != 0) nrm = 0.0;
        if (slot) nrm = nrm + slot_residual_norm_x16(P, z, Uown, color ^ 1, t, lane);
        residual_partial(res_partial, xb, nrm);
    }
    const bool stop = stop_decision(st, share);
    if (!cell || lane != 0 || stop || (gate && flag_set(gate))) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) Uout[c * N + idx] = q[c];
}

// Relaxed update U += tau_i dU (positivity-limited tau_i) and dry threshold.
template <int NC, class T>
__device__ __forceinline__ void update_cell(const Phys &P, const LevelGeom &G,
                                            const T *__restrict__ x, double *__restrict__ U,
                                            long idx)
{
    const long N = (long)P.nx * P.ny;
    int i = (int)(idx % P.nx), j = (int)(idx / P.nx);
    const int color = (i + j) & 1;
    const T *xs = x + (long)color * NC * G.plane + (long)j * G.W + (i >> 1);
    double dq[NC], q[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        dq[c] = double(xs[c * G.plane]);
        q[c] = U[c * N + idx];
    }
    const double th = P.pos_theta, tau = P.tau;
    double t = tau;
    double h = q[0], dh = dq[0];
    if (th > 0.0 && dh < 0.0 && h + tau * dh < (1.0 - th) * h) t = th * h / (-dh);
#pragma unroll
    for (int c = 0; c < NC; ++c) q[c] = q[c] + t * dq[c];
    if (q[0] < P.h_eps) {
#pragma unroll
        for (int c = 0; c < NC; ++c) q[c] = 0.0;
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) U[c * N + idx] = q[c];
}

template <int NC, class T>
__global__ void __launch_bounds__(kBlock) k_update(Phys P, LevelGeom G,
                                                   const T *__restrict__ x,
                                                   double *__restrict__ U)
{
    long idx = (long)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (long)P.nx * P.ny) return;
    update_cell<NC, T>(P, G, x, U, idx);
}

template <int NC>
__device__ __forceinline__ void threshold_cell(const Phys &P, double *__restrict__ U, long idx)
{
    const long N = (long)P.nx * P.ny;
    if (U[idx] < P.h_eps) {
#pragma unroll
        for (int c = 0; c < NC; ++c) U[c * N + idx] = 0.0;
    }
}

template <int NC>
__global__ void __launch_bounds__(kBlock) k_threshold(Phys P, double *__restrict__ U)
{
    long idx = (long)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (long)P.nx * P.ny) return;
    threshold_cell<NC>(P, U, idx);
}

// ---------------------------------------------------------------------------
// Linear multigrid kernels on the colour-split layout.

// Linear residual of fine cell (i, j): b - (D x_i + sum_nbr A x_nbr).
// STREAM: off-diagonal blocks loaded through ld_once (read once per launch).
template <class T, int NC, bool STREAM = false>
__device__ __forceinline__ void lin_residual_cell(const LevelGeom &G, const T *A,
                                                  const T *b, const T *x, int i, int j,
                                                  T *r)
{
    const int NF = (NC == 2) ? 2 : 4;
    const int NE = (NF + 1) * NC * NC;
    const int color = (i + j) & 1;
    const long slot = (long)j * G.W + (i >> 1);
    const T *Am = A + mat_off(G, NE, color, slot);
    const T *bm = b + (long)color * NC * G.plane + slot;
    const T *xm = x + (long)color * NC * G.plane + slot;
    const T *xo = x + (long)(color ^ 1) * NC * G.plane;
    T xi[NC], acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) xi[c] = xm[c * G.plane];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        acc[q] = T(0);
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[q] = acc[q] + Am[(q * NC + c) * kTile] * xi[c];
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        int ni = i, nj = j;
        bool ok;
        if (f == FW) { ni = i - 1; ok = i > 0; }
        else if (f == FE) { ni = i + 1; ok = i + 1 < G.nx; }
        else if (f == FS) { nj = j - 1; ok = j > 0; }
        else { nj = j + 1; ok = j + 1 < G.ny; }
        if (!ok) continue;
        const T *p = xo + (long)nj * G.W + (ni >> 1);
        T v[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = p[c * G.plane];
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int c = 0; c < NC; ++c)
                acc[q] = acc[q] + ld_once<T, STREAM>(&Am[(((f + 1) * NC + q) * NC + c) * kTile]) * v[c];
    }
#pragma unroll
    for (int q = 0; q < NC; ++q) r[q] = bm[q * G.plane] - acc[q];
}

// Restriction (eq:ProjectAR, right): coarse right-hand side = sum over the
// children (SW, SE, NW, NE; 1D: left, right) of their linear residuals.
template <class T, int NC>
__device__ __forceinline__ void restrict_cell(const LevelGeom &G, const T *__restrict__ A,
                                              const T *__restrict__ b,
                                              const T *__restrict__ x, const LevelGeom &Gc,
                                              T *__restrict__ bc, long t)
{
    const int I = (int)(t % Gc.nx), J = (int)(t / Gc.nx);
    const int nch = (NC == 2) ? 2 : 4;
    T acc[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) acc[q] = T(0);
#pragma unroll
    for (int ch = 0; ch < nch; ++ch) {
        int i = 2 * I + (ch & 1);
        int j = (NC == 2) ? 0 : 2 * J + (ch >> 1);
        T r[NC];
        lin_residual_cell<T, NC>(G, A, b, x, i, j, r);
#pragma unroll
        for (int q = 0; q < NC; ++q) acc[q] = acc[q] + r[q];
    }
    const int cc = (I + J) & 1;
    T *bm = bc + (long)cc * NC * Gc.plane + (long)J * Gc.W + (I >> 1);
#pragma unroll
    for (int q = 0; q < NC; ++q) bm[q * Gc.plane] = acc[q];
}

// Restriction with one thread per child: a block of kBlock threads covers
// CB = kBlock / nch consecutive coarse cells (nch = 4 children in 2D, 2 in
// 1D); thread u of the block handles child u / CB of cell u % CB, so each
// wave reads one child position of consecutive cells (coalesced), and the
// block's first CB threads sum the children's residuals, exchanged through
// LDS, in the order of restrict_cell.  base: index of the block's first
// coarse cell.  Every thread of the block reaches the barrier.
// RIN: the residuals of the children of colour rcol were written by the half
// sweep that last updated them (k_sgs_half_res, NC planes of that colour's
// slots in rin) and are read instead of recomputed; a child position has
// one colour, so each wave either reads or computes.
template <class T, int NC, bool STREAM = false, bool RIN = false>
__device__ __forceinline__ void restrict_block(const LevelGeom &G, const T *__restrict__ A,
                                               const T *__restrict__ b,
                                               const T *__restrict__ x, const LevelGeom &Gc,
                                               T *__restrict__ bc, long base,
                                               const T *__restrict__ rin = nullptr, int rcol = 0)
{
    constexpr int nch = (NC == 2) ? 2 : 4;
    constexpr int CB = kBlock / nch;
    __shared__ T rs[nch][NC][CB];
    const int ch = (int)threadIdx.x / CB, k = (int)threadIdx.x % CB;
    const long t = base + k;
    const bool valid = t < (long)Gc.nx * Gc.ny;
    const int I = valid ? (int)(t % Gc.nx) : 0, J = valid ? (int)(t / Gc.nx) : 0;
    if (valid) {
        T r[NC];
        const int i = 2 * I + (ch & 1);
        const int j = (NC == 2) ? 0 : 2 * J + (ch >> 1);
        if (RIN && ((i + j) & 1) == rcol) {
            const long slot = (long)j * G.W + (i >> 1);
#pragma unroll
            for (int q = 0; q < NC; ++q) r[q] = rin[q * G.plane + slot];
        } else {
            lin_residual_cell<T, NC, STREAM>(G, A, b, x, i, j, r);
        }
#pragma unroll
        for (int q = 0; q < NC; ++q) rs[ch][q][k] = r[q];
    }
    __syncthreads();
    if (valid && ch == 0) {
        T acc[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) acc[q] = T(0);
#pragma unroll
        for (int c = 0; c < nch; ++c)
#pragma unroll
            for (int q = 0; q < NC; ++q) acc[q] = acc[q] + rs[c][q][k];
        const int cc = (I + J) & 1;
        T *bm = bc + (long)cc * NC * Gc.plane + (long)J * Gc.W + (I >> 1);
#pragma unroll
        for (int q = 0; q < NC; ++q) bm[q * Gc.plane] = acc[q];
    }
}

template <class T, int NC, bool STREAM>
__global__ void __launch_bounds__(kBlock) k_restrict(LevelGeom G, const T *__restrict__ A,
                                                     const T *__restrict__ b,
                                                     const T *__restrict__ x, LevelGeom Gc,
                                                     T *__restrict__ bc)
{
    const int xb = xcd_block(blockIdx.x, gridDim.x);
    restrict_block<T, NC, STREAM>(G, A, b, x, Gc, bc, (long)xb * (kBlock / ((NC == 2) ? 2 : 4)));
}

template <class T, int NC, bool STREAM>
__global__ void __launch_bounds__(kBlock) k_restrict_res(LevelGeom G, const T *__restrict__ A,
                                                         const T *__restrict__ b,
                                                         const T *__restrict__ x, LevelGeom Gc,
                                                         T *__restrict__ bc,
                                                         const T *__restrict__ rin, int rcol)
{
    const int xb = xcd_block(blockIdx.x, gridDim.x);
    restrict_block<T, NC, STREAM, true>(G, A, b, x, Gc, bc,
                                        (long)xb * (kBlock / ((NC == 2) ? 2 : 4)), rin, rcol);
}

// Galerkin coarse blocks (eq:ProjectAR, left) with the child-pair order of
// the definition: children of I (SW, SE, NW, NE), then children of J.
// STREAM: the fine blocks (each read once) are loaded with the non-temporal
// hint.
template <class T, int NC, bool STREAM = false>
__device__ __forceinline__ void galerkin_cell(const LevelGeom &Gf, const T *__restrict__ Af,
                                              const LevelGeom &Gc, T *__restrict__ Ac, long t)
{
    const int NF = (NC == 2) ? 2 : 4;
    const int NE = (NF + 1) * NC * NC;
    const int NN = NC * NC;
    const int I = (int)(t % Gc.nx), J = (int)(t / Gc.nx);
    // child (ci, cj) block blk entry e -> pointer
    auto ent = [&](int ci, int cj, int blk, int e) -> T {
        int col = (ci + cj) & 1;
        const T *p = &Af[mat_off(Gf, NE, col, (long)cj * Gf.W + (ci >> 1)) + (blk * NN + e) * kTile];
        if constexpr (STREAM) return __builtin_nontemporal_load(p);
        else return *p;
    };
    const int cc = (I + J) & 1;
    T *out = Ac + mat_off(Gc, NE, cc, (long)J * Gc.W + (I >> 1));
    enum { BD = 0, BW = 1, BE = 2, BS = 3, BN = 4 };
    if (NC == 2) {
        const int L = 2 * I, R = 2 * I + 1;
        for (int e = 0; e < NN; ++e) {
            T d = T(0);
            d = d + ent(L, 0, BD, e);
            d = d + ent(L, 0, BE, e);
            d = d + ent(R, 0, BW, e);
            d = d + ent(R, 0, BD, e);
            out[(BD * NN + e) * kTile] = d;
            T w = T(0), ea = T(0);
            if (I > 0) w = w + ent(L, 0, BW, e);
            if (I + 1 < Gc.nx) ea = ea + ent(R, 0, BE, e);
            out[(BW * NN + e) * kTile] = w;
            out[(BE * NN + e) * kTile] = ea;
        }
        return;
    }
    const int x0 = 2 * I, x1 = 2 * I + 1, y0 = 2 * J, y1 = 2 * J + 1;
    for (int e = 0; e < NN; ++e) {
        T d = T(0);
        d = d + ent(x0, y0, BD, e);   // SW -> SW
        d = d + ent(x0, y0, BE, e);   // SW -> SE
        d = d + ent(x0, y0, BN, e);   // SW -> NW
        d = d + ent(x1, y0, BW, e);   // SE -> SW
        d = d + ent(x1, y0, BD, e);   // SE -> SE
        d = d + ent(x1, y0, BN, e);   // SE -> NE
        d = d + ent(x0, y1, BS, e);   // NW -> SW
        d = d + ent(x0, y1, BD, e);   // NW -> NW
        d = d + ent(x0, y1, BE, e);   // NW -> NE
        d = d + ent(x1, y1, BS, e);   // NE -> SE
        d = d + ent(x1, y1, BW, e);   // NE -> NW
        d = d + ent(x1, y1, BD, e);   // NE -> NE
        out[(BD * NN + e) * kTile] = d;
        T w = T(0), ea = T(0), s = T(0), n = T(0);
        if (I > 0) { w = w + ent(x0, y0, BW, e); w = w + ent(x0, y1, BW, e); }
        if (I + 1 < Gc.nx) { ea = ea + ent(x1, y0, BE, e); ea = ea + ent(x1, y1, BE, e); }
        if (J > 0) { s = s + ent(x0, y0, BS, e); s = s + ent(x1, y0, BS, e); }
        if (J + 1 < Gc.ny) { n = n + ent(x0, y1, BN, e); n = n + ent(x1, y1, BN, e); }
        out[(BW * NN + e) * kTile] = w;
        out[(BE * NN + e) * kTile] = ea;
        out[(BS * NN + e) * kTile] = s;
        out[(BN * NN + e) * kTile] = n;
    }
}

template <class T, int NC, bool STREAM = false>
__global__ void __launch_bounds__(kBlock) k_galerkin(LevelGeom Gf, const T *__restrict__ Af,
                                                     LevelGeom Gc, T *__restrict__ Ac)
{
    long t = (long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (long)Gc.nx * Gc.ny) return;
    galerkin_cell<T, NC, STREAM>(Gf, Af, Gc, Ac, t);
}

template <class T, int NC>
__device__ __forceinline__ void fix_cell(const LevelGeom &G, int op, T *__restrict__ x,
                                         int color, const LevelGeom &Gc,
                                         const T *__restrict__ xc, long t)
{
    const int j = (int)(t / G.W), k = (int)(t % G.W);
    const int i = 2 * k + ((j + color) & 1);
    if (i >= G.nx) return;
    T *xm = x + (long)color * NC * G.plane + t;
    if (op == 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) xm[c * G.plane] = T(0);
        return;
    }
    int I = i >> 1, J = j >> 1;
    int cc = (I + J) & 1;
    const T *p = xc + (long)cc * NC * Gc.plane + (long)J * Gc.W + (I >> 1);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        T base = (op == 1) ? xm[c * G.plane] : T(0);
        xm[c * G.plane] = base + p[c * Gc.plane];
    }
}

template <class T, int NC>
__global__ void __launch_bounds__(kBlock) k_fix_color(LevelGeom G, int op, T *__restrict__ x,
                                                      int color, LevelGeom Gc,
                                                      const T *__restrict__ xc)
{
    long t = (long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= G.plane) return;
    fix_cell<T, NC>(G, op, x, color, Gc, xc, t);
}

// A pointer known to address global memory.  Its bits are taken as a
// global-address-space pointer (a global address is the same value in the
// generic space) and converted back, so the compiler uses global (not
// generic) loads and stores for everything derived from it.  A plain cast
// to the global space and back is folded away and leaves generic accesses,
// whose completion the LDS wait counter also tracks.
template <class T>
__device__ __forceinline__ T *in_global(T *p)
{
    __attribute__((address_space(1))) void *g;
    __builtin_memcpy(&g, &p, sizeof(g));
    return (T *)g;
}

// A batch level entry with its arrays as global pointers (in_global).
__device__ __forceinline__ BatchLevel global_view(const BatchLevel &L)
{
    BatchLevel J = L;
    J.A = in_global(L.A);
    J.b = in_global(L.b);
    J.x = in_global(L.x);
    J.Ac = in_global(L.Ac);
    J.bc = in_global(L.bc);
    J.xc = in_global(L.xc);
    J.xt = in_global(L.xt);
    J.rr = in_global(L.rr);
    return J;
}

// One recorded operation on level G (blocks A, inverse data Ai when INV,
// vectors b, x) with the next coarser level's b and x (bc, xc).
template <class T, int NC, bool INV>
__device__ __forceinline__ void coarse_op(const CoarseOp &op, const LevelGeom &G,
                                          const LevelGeom &Gc, const T *A, const T *Ai, const T *b,
                                          T *x, T *bc, const T *xc)
{
    if (op.kind == COP_SGS) {
        for (long t = threadIdx.x; t < G.plane; t += kCoarseBlock) {
            switch (op.mode) {
            case MODE_NORMAL:
                sgs_cell<T, NC, MODE_NORMAL, INV>(G, A, Ai, b, x, op.color, Gc, xc, t);
                break;
            case MODE_ZERO:
                sgs_cell<T, NC, MODE_ZERO, INV>(G, A, Ai, b, x, op.color, Gc, xc, t);
                break;
            case MODE_PROLONG:
                sgs_cell<T, NC, MODE_PROLONG, INV>(G, A, Ai, b, x, op.color, Gc, xc, t);
                break;
            default:
                sgs_cell<T, NC, MODE_PROLONG_ZERO, INV>(G, A, Ai, b, x, op.color, Gc, xc, t);
                break;
            }
        }
    } else if (op.kind == COP_RESTRICT) {
        for (long t = threadIdx.x; t < (long)Gc.nx * Gc.ny; t += kCoarseBlock)
            restrict_cell<T, NC>(G, A, b, x, Gc, bc, t);
    } else {
        for (long t = threadIdx.x; t < G.plane; t += kCoarseBlock)
            fix_cell<T, NC>(G, op.mode, x, op.color, Gc, xc, t);
    }
}

// A run of op.count alternating half sweeps on an LDS-resident level whose
// cells all have a thread (2 * plane <= kCoarseBlock): colour op.color ^ (s & 1)
// at step s, the first in op.mode (normal or zero start), the rest normal.
// Each thread keeps its cell's off-diagonal blocks, block inverse and
// right-hand side in registers for the whole run, so a half sweep is the
// neighbour reads, the update and one write of x, all in LDS.
template <class T, int NC>
__device__ __forceinline__ void coarse_run(const CoarseOp &op, const LevelGeom &G, const T *A,
                                           const T *Ai, const T *b, T *x)
{
    constexpr int NF = (NC == 2) ? 2 : 4;
    constexpr int NN = NC * NC;
    constexpr int NE = (NF + 1) * NN;
    constexpr int NI = inv_entries(NC);
    const int plane = (int)G.plane;
    const int tau = (int)threadIdx.x;
    const int color = tau < plane ? 0 : 1;
    const int t = tau - color * plane;
    const int j = t / G.W, k = t - (t / G.W) * G.W;
    const int i = 2 * k + ((j + color) & 1);
    const bool mine = tau < 2 * plane && i < G.nx;
    bool ok[NF];
    int nb[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        int ni = i, nj = j;
        if (f == FW) { ni = i - 1; ok[f] = i > 0; }
        else if (f == FE) { ni = i + 1; ok[f] = i + 1 < G.nx; }
        else if (f == FS) { nj = j - 1; ok[f] = j > 0; }
        else { nj = j + 1; ok[f] = j + 1 < G.ny; }
        nb[f] = nj * G.W + (ni >> 1);
    }
    T a[NE], inv[NI], bv[NC];
    if (mine) {
        const T *Am = A + mat_off(G, NE, color, t);
        const T *Im = Ai + mat_off(G, NI, color, t);
#pragma unroll
        for (int e = NN; e < NE; ++e) a[e] = Am[e * kTile];
#pragma unroll
        for (int e = 0; e < NI; ++e) inv[e] = Im[e * kTile];
#pragma unroll
        for (int r = 0; r < NC; ++r) bv[r] = b[(color * NC + r) * plane + t];
    }
    const T *xo = x + (color ^ 1) * NC * plane;
    T *xm = x + color * NC * plane + t;
    for (int s = 0; s < op.count; ++s) {
        if (mine && color == (op.color ^ (s & 1))) {
            T v[NF][NC], xi[NC];
            if (s == 0 && op.mode == MODE_ZERO) {
                gs_update<T, NC, true, true>(a, inv, bv, v, ok, xi);
            } else {
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const int q = ok[f] ? nb[f] : t;      // a valid slot; its value is dropped
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        const T val = xo[c * plane + q];
                        v[f][c] = ok[f] ? val : T(0);
                    }
                }
                gs_update<T, NC, false, true>(a, inv, bv, v, ok, xi);
            }
#pragma unroll
            for (int r = 0; r < NC; ++r) xm[r * plane] = xi[r];
        }
        if (s + 1 < op.count) __syncthreads();
    }
}

// Exchange a value with the neighbouring lane of the pair (lanes 2m, 2m+1).
template <class T>
__device__ __forceinline__ T swap_pair(T v)
{
    constexpr int kSwap = 0xB1;     // quad_perm [1, 0, 3, 2]
    if constexpr (sizeof(T) == 8) {
        const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
        const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)u, kSwap, 0xF, 0xF, false);
        const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), kSwap, 0xF, 0xF, false);
        return __builtin_bit_cast(T, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
    } else {
        return __builtin_bit_cast(T, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), kSwap,
                                                              0xF, 0xF, false));
    }
}

// coarse_run for 3x3 blocks with two lanes per cell (4 * plane <= kCoarseBlock):
// lane 0 of a pair sums rows 0 and 1 of b_i - sum_j A_ij x_j, lane 1 row 2
// (its second row is a zero row that nothing reads); the pair swaps the
// three right-hand sides and each lane applies its rows of the inverse data.
// A half sweep then occupies twice as many waves with about half the
// instructions each, so all four SIMDs share it.  Every row's sum, the
// right-hand side and the products with the inverse data are the
// operations of gs_update and solve_inv in their order, so the result is
// bit for bit that of coarse_run.  A missing face reads the zero at zslot
// instead of selecting zero.
template <class T>
__device__ __forceinline__ void coarse_run_split(const CoarseOp &op, const LevelGeom &G,
                                                 const T *A, const T *Ai, const T *b, T *x,
                                                 const T *zslot)
{
    constexpr int NC = 3, NF = 4, NN = 9, NE = 45, NI = inv_entries(3);
    const int plane = (int)G.plane;
    const int tau = (int)threadIdx.x >> 1, h = (int)threadIdx.x & 1;
    const int color = tau < plane ? 0 : 1;
    const int t = tau - color * plane;
    const int j = t / G.W, k = t - (t / G.W) * G.W;
    const int i = 2 * k + ((j + color) & 1);
    const bool mine = tau < 2 * plane && i < G.nx;
    const T *xo = x + (color ^ 1) * NC * plane;
    const T *src[NF][NC];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        int ni = i, nj = j;
        bool ok;
        if (f == FW) { ni = i - 1; ok = i > 0; }
        else if (f == FE) { ni = i + 1; ok = i + 1 < G.nx; }
        else if (f == FS) { nj = j - 1; ok = j > 0; }
        else { nj = j + 1; ok = j + 1 < G.ny; }
        const int q = nj * G.W + (ni >> 1);
#pragma unroll
        for (int c = 0; c < NC; ++c) src[f][c] = ok ? xo + c * plane + q : zslot;
    }
    // this lane's rows: 2h and (h == 0 only) 1
    T a[2][NF * NC], inv[2][NC], bv[2], idet = T(0);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
#pragma unroll
        for (int e = 0; e < NF * NC; ++e) a[r][e] = T(0);
#pragma unroll
        for (int c = 0; c < NC; ++c) inv[r][c] = T(0);
        bv[r] = T(0);
    }
    if (mine) {
        const T *Am = A + mat_off(G, NE, color, t);
        const T *Im = Ai + mat_off(G, NI, color, t);
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int row = r == 0 ? 2 * h : 1;
            if (r == 1 && h) break;
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    a[r][f * NC + c] = Am[(((f + 1) * NC + row) * NC + c) * kTile];
#pragma unroll
            for (int c = 0; c < NC; ++c) inv[r][c] = Im[(NC * row + c) * kTile];
            bv[r] = b[(color * NC + row) * plane + t];
        }
        idet = Im[NN * kTile];
    }
    const bool sing = idet != idet;
    T *xm = x + color * NC * plane + t;
    for (int s = 0; s < op.count; ++s) {
        if (mine && color == (op.color ^ (s & 1))) {
            T acc[2] = {T(0), T(0)};
            if (!(s == 0 && op.mode == MODE_ZERO)) {
                T v[NF][NC];
#pragma unroll
                for (int f = 0; f < NF; ++f)
#pragma unroll
                    for (int c = 0; c < NC; ++c) v[f][c] = *src[f][c];
                // all twelve reads in flight before the arithmetic (one LDS
                // round trip instead of the scheduler's three)
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    T p[2][NC];
#pragma unroll
                    for (int r = 0; r < 2; ++r)
#pragma unroll
                        for (int c = 0; c < NC; ++c) p[r][c] = a[r][f * NC + c] * v[f][c];
#pragma unroll
                    for (int c = 0; c < NC; ++c)
#pragma unroll
                        for (int r = 0; r < 2; ++r) acc[r] = acc[r] + p[r][c];
                }
            }
            const T own0 = bv[0] - acc[0], own1 = bv[1] - acc[1];
            const T oth0 = swap_pair(own0), oth1 = swap_pair(own1);
            const T r0 = h ? oth0 : own0, r1 = h ? oth1 : own1, r2 = h ? own0 : oth0;
            T xr[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                xr[r] = (inv[r][0] * r0 + inv[r][1] * r1 + inv[r][2] * r2) * idet;
                xr[r] = sing ? T(0) : xr[r];
            }
            xm[2 * h * plane] = xr[0];
            if (!h) xm[plane] = xr[1];
        }
        if (s + 1 < op.count) __syncthreads();
    }
}

// One cell of a register-resident run: the cell of colour `color` at slot
// threadIdx.x of a level in global memory (if it exists), its off-diagonal
// blocks and the inverse data of its diagonal block (block_inverse), loaded
// once for the whole run.  Its neighbours, right-hand side and (for the
// residual) diagonal block are recomputed or reloaded where used, which
// keeps two cells per thread within the register file.
template <class T, int NC>
struct RegCell {
    static constexpr int NF = (NC == 2) ? 2 : 4;
    static constexpr int NN = NC * NC;
    static constexpr int NE = (NF + 1) * NN;
    static constexpr int NI = inv_entries(NC);
    bool mine;
    T a[NE];          // a[0, NN) unused; a[NN, NE) the off-diagonal blocks
    T inv[NI];

    __device__ __forceinline__ static void where(const LevelGeom &G, int color, int t, int &i,
                                                 int &j)
    {
        j = t / G.W;
        i = 2 * (t - j * G.W) + ((j + color) & 1);
    }
    __device__ __forceinline__ static void face(const LevelGeom &G, int i, int j, int f, int &ni,
                                                int &nj, bool &ok)
    {
        ni = i;
        nj = j;
        if (f == FW) { ni = i - 1; ok = i > 0; }
        else if (f == FE) { ni = i + 1; ok = i + 1 < G.nx; }
        else if (f == FS) { nj = j - 1; ok = j > 0; }
        else { nj = j + 1; ok = j + 1 < G.ny; }
    }

    __device__ __forceinline__ void load(const LevelGeom &G, const T *A, int color, int t)
    {
        int i, j;
        where(G, color, t, i, j);
        mine = t < G.plane && i < G.nx;
        if (mine) {
            const T *Am = in_global(A) + mat_off(G, NE, color, t);
            T D[NN];
#pragma unroll
            for (int e = 0; e < NN; ++e) D[e] = Am[e * kTile];
#pragma unroll
            for (int e = NN; e < NE; ++e) a[e] = Am[e * kTile];
            block_inverse<T, NC>(D, inv);
        }
    }

    // Half sweep update of this cell: the arithmetic of sgs_cell (solve_inv
    // with block_inverse's data is solve_block bit for bit).
    template <int MODE>
    __device__ __forceinline__ void update(const LevelGeom &G, const T *b, T *x, int color,
                                           const LevelGeom &Gc, const T *xc, int t) const
    {
        if (!mine) return;
        int i, j;
        where(G, color, t, i, j);
        const T *xo = x + (long)(color ^ 1) * NC * G.plane;
        T v[NF][NC], xi[NC], bv[NC];
        bool ok[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            int ni, nj;
            face(G, i, j, f, ni, nj, ok[f]);
            if (MODE != MODE_ZERO) {
                if (ok[f]) {
                    read_other<T, NC, MODE>(G, xo, ni, nj, Gc, xc, v[f]);
                } else {
#pragma unroll
                    for (int c = 0; c < NC; ++c) v[f][c] = T(0);
                }
            }
        }
        const T *bg = in_global(b);
#pragma unroll
        for (int r = 0; r < NC; ++r) bv[r] = bg[((long)color * NC + r) * G.plane + t];
        gs_update<T, NC, MODE == MODE_ZERO, true>(a, inv, bv, v, ok, xi);
        T *xm = x + (long)color * NC * G.plane + t;
#pragma unroll
        for (int r = 0; r < NC; ++r) xm[r * G.plane] = xi[r];
    }

    __device__ __forceinline__ void first(int mode, const LevelGeom &G, const T *b, T *x,
                                          int color, const LevelGeom &Gc, const T *xc,
                                          int t) const
    {
        switch (mode) {
        case MODE_NORMAL: update<MODE_NORMAL>(G, b, x, color, Gc, xc, t); break;
        case MODE_ZERO: update<MODE_ZERO>(G, b, x, color, Gc, xc, t); break;
        case MODE_PROLONG: update<MODE_PROLONG>(G, b, x, color, Gc, xc, t); break;
        default: update<MODE_PROLONG_ZERO>(G, b, x, color, Gc, xc, t); break;
        }
    }

    // Linear residual r of this cell: the arithmetic of lin_residual_cell,
    // with the diagonal block reloaded from A.
    __device__ __forceinline__ void residual(const LevelGeom &G, const T *A, const T *b,
                                             const T *x, int color, int t, T *r) const
    {
        int i, j;
        where(G, color, t, i, j);
        const T *Am = in_global(A) + mat_off(G, NE, color, t);
        const T *bg = in_global(b);
        const T *xm = x + (long)color * NC * G.plane + t;
        const T *xo = x + (long)(color ^ 1) * NC * G.plane;
        T xi[NC], acc[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) xi[c] = xm[c * G.plane];
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            acc[q] = T(0);
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[q] = acc[q] + Am[(q * NC + c) * kTile] * xi[c];
        }
        // every face's values are read at once (a missing face reads a valid
        // slot and takes zero); a missing face has a zero block, so its +0
        // terms leave acc as lin_residual_cell's skipped face does (acc
        // starts at +0 and never becomes -0)
        T v[NF][NC];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            int ni, nj;
            bool ok;
            face(G, i, j, f, ni, nj, ok);
            const long q = ok ? (long)nj * G.W + (ni >> 1) : (long)t;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const T val = xo[c * G.plane + q];
                v[f][c] = ok ? val : T(0);
            }
        }
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int q = 0; q < NC; ++q)
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    acc[q] = acc[q] + a[((f + 1) * NC + q) * NC + c] * v[f][c];
#pragma unroll
        for (int q = 0; q < NC; ++q) r[q] = bg[((long)color * NC + q) * G.plane + t] - acc[q];
    }
};

// COP_REGRUN: op.count alternating half sweeps on a level in global memory
// with at most one slot per colour and thread (the first in op.mode, the
// rest normal), each thread holding the block rows of its red and its black
// cell in registers, so the level's blocks are read once per run instead of
// once per half sweep.  x moves to the LDS area xl (2 NC plane values) for
// the run and back afterwards.  Then, if op.aux, the restriction to the next
// level: restrict_cell's sums in its child order, the children's residuals
// exchanged through the same LDS area.  The caller's barrier follows.
template <class T, int NC>
__device__ __forceinline__ void reg_run_body(const CoarseOp &op, const LevelGeom &G,
                                             const T *A, const T *b, T *x, const LevelGeom &Gc,
                                             T *bc, const T *xc, T *xl,
                                             const RegCell<T, NC> &red,
                                             const RegCell<T, NC> &black);

// KEEP: the block rows live in *keep (loaded by the first run of the
// program, *loaded set); otherwise they are loaded here for this run.
template <class T, int NC, bool KEEP>
__device__ __forceinline__ void coarse_reg_run(const CoarseOp &op, const LevelGeom &G,
                                               const T *A, const T *b, T *x, const LevelGeom &Gc,
                                               T *bc, const T *xc, T *xl, RegCell<T, NC> *keep,
                                               bool *loaded)
{
    const int t = (int)threadIdx.x;
    const int nv = 2 * NC * (int)G.plane;
    for (int k = t; k < nv; k += kCoarseBlock) xl[k] = x[k];
    if constexpr (KEEP) {
        if (!*loaded) {
            keep[0].load(G, A, 0, t);
            keep[1].load(G, A, 1, t);
            *loaded = true;
        }
        __syncthreads();
        reg_run_body<T, NC>(op, G, A, b, x, Gc, bc, xc, xl, keep[0], keep[1]);
    } else {
        RegCell<T, NC> red, black;
        red.load(G, A, 0, t);
        black.load(G, A, 1, t);
        __syncthreads();
        reg_run_body<T, NC>(op, G, A, b, x, Gc, bc, xc, xl, red, black);
    }
}

template <class T, int NC>
__device__ __forceinline__ void reg_run_body(const CoarseOp &op, const LevelGeom &G,
                                             const T *A, const T *b, T *x, const LevelGeom &Gc,
                                             T *bc, const T *xc, T *xl,
                                             const RegCell<T, NC> &red,
                                             const RegCell<T, NC> &black)
{
    const int t = (int)threadIdx.x;
    const int nv = 2 * NC * (int)G.plane;
    if (op.color == 0) red.first(op.mode, G, b, xl, 0, Gc, xc, t);
    else black.first(op.mode, G, b, xl, 1, Gc, xc, t);
    __syncthreads();
    for (int s = 1; s < op.count; ++s) {
        if ((op.color ^ (s & 1)) == 0) red.template update<MODE_NORMAL>(G, b, xl, 0, Gc, xc, t);
        else black.template update<MODE_NORMAL>(G, b, xl, 1, Gc, xc, t);
        __syncthreads();
    }
    T rr[NC], rb[NC];
    if (op.aux) {
        if (red.mine) red.residual(G, A, b, xl, 0, t, rr);
        if (black.mine) black.residual(G, A, b, xl, 1, t, rb);
    }
    for (int k = t; k < nv; k += kCoarseBlock) x[k] = xl[k];
    if (!op.aux) return;
    __syncthreads();
    T *rs = xl;
    const int plane = (int)G.plane;
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        if (red.mine) rs[q * plane + t] = rr[q];
        if (black.mine) rs[(NC + q) * plane + t] = rb[q];
    }
    __syncthreads();
    const int nch = (NC == 2) ? 2 : 4;
    for (int u = t; u < Gc.nx * Gc.ny; u += kCoarseBlock) {
        const int I = u % Gc.nx, J = u / Gc.nx;
        T acc[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) acc[q] = T(0);
#pragma unroll
        for (int ch = 0; ch < nch; ++ch) {
            const int i = 2 * I + (ch & 1);
            const int j = (NC == 2) ? 0 : 2 * J + (ch >> 1);
            const int col = (i + j) & 1;
            const int slot = j * G.W + (i >> 1);
#pragma unroll
            for (int q = 0; q < NC; ++q) acc[q] = acc[q] + rs[(col * NC + q) * plane + slot];
        }
        const int cc = (I + J) & 1;
        T *bm = bc + (long)cc * NC * Gc.plane + (long)J * Gc.W + (I >> 1);
#pragma unroll
        for (int q = 0; q < NC; ++q) bm[q * Gc.plane] = acc[q];
    }
}

// Pointers into a level's LDS copy (layout of LevelDev::lds_off).
template <class T, int NC>
struct LdsLevel {
    T *A, *Ai, *b, *x;
    __device__ __forceinline__ LdsLevel(char *lds, const LevelDev &L)
    {
        constexpr int NE = ((NC == 2) ? 3 : 5) * NC * NC;
        A = (T *)(lds + L.lds_off);
        Ai = A + 2L * NE * L.G.planeP;
        b = Ai + 2L * inv_entries(NC) * L.G.planeP;
        x = b + 2L * NC * L.G.plane;
    }
};

// COP_REGRUN on level Ld (global) with the next level Lc (LDS or global).
template <class T, int NC, bool KEEP>
__device__ __forceinline__ void coarse_reg_level(const CoarseOp &op, const LevelDev &Ld,
                                                 const LevelDev &Lc, char *lds,
                                                 RegCell<T, NC> *keep, bool *loaded)
{
    T *xl = (T *)(lds + op.lds_off);
    if (Lc.lds_off >= 0) {
        const LdsLevel<T, NC> Cl(lds, Lc);
        coarse_reg_run<T, NC, KEEP>(op, Ld.G, in_global((const T *)Ld.A),
                                    in_global((const T *)Ld.b), in_global((T *)Ld.x), Lc.G, Cl.b,
                                    Cl.x, xl, keep, loaded);
    } else {
        coarse_reg_run<T, NC, KEEP>(op, Ld.G, in_global((const T *)Ld.A),
                                    in_global((const T *)Ld.b), in_global((T *)Ld.x), Lc.G,
                                    in_global((T *)Lc.b), in_global((const T *)Lc.x), xl, keep,
                                    loaded);
    }
}

// The coarse levels of a cycle in one workgroup: the host records the exact
// sequence of half sweeps, restrictions and colour fixes that the
// level-by-level launches would perform, and this kernel executes it with a
// workgroup barrier between operations.  The coarsest levels (those with
// lds_off >= 0) are first copied into LDS together with their blocks'
// inverse data, so their many half sweeps run at LDS latency without a
// division; their vectors are copied back at the end.  Every pointer is
// formed in the branch that uses it, from the LDS array or from the level
// table, so each access compiles to an LDS or a global load, never a generic
// one.  The operation list and level table are read with uniform loads.
//
// In a batch, workgroup k runs instance k with the level table
// lv + k * kMaxLevels and does nothing if active[k] is 0.
template <class T, int NC>
__global__ void __launch_bounds__(kCoarseBlock) k_coarse_cycle(const CoarseOp *__restrict__ ops,
                                                               int nops,
                                                               const LevelDev *__restrict__ lv,
                                                               const int *__restrict__ active,
                                                               int l_lds, int nl)
{
    constexpr int NF = (NC == 2) ? 2 : 4;
    constexpr int NN = NC * NC;
    constexpr int NE = (NF + 1) * NN;
    constexpr int NI = inv_entries(NC);
    __shared__ __attribute__((aligned(16))) char lds[kCoarseLdsBytes];
    __shared__ T zslot[1];       // a zero that split runs read for missing faces
    if (active && !active[blockIdx.x]) return;
    lv += (long)blockIdx.x * kMaxLevels;
    if (l_lds >= 0) {
        if (threadIdx.x == 0) zslot[0] = T(0);
        for (int l = l_lds; l <= nl; ++l) {
            const LevelDev &L = lv[l];
            const LdsLevel<T, NC> S(lds, L);
            const long na = 2L * NE * L.G.planeP, nv = 2L * NC * L.G.plane;
            const T *gA = in_global((const T *)L.A), *gb = in_global((const T *)L.b);
            const T *gx = in_global((const T *)L.x);
            for (long k = threadIdx.x; k < na; k += kCoarseBlock) S.A[k] = gA[k];
            for (long k = threadIdx.x; k < nv; k += kCoarseBlock) { S.b[k] = gb[k]; S.x[k] = gx[k]; }
            for (long k = threadIdx.x; k < 2L * L.G.planeP; k += kCoarseBlock) {
                const int color = (int)(k / L.G.planeP);
                const long t = k % L.G.planeP;
                const T *Dm = gA + mat_off(L.G, NE, color, t);
                T D[NN], inv[NI];
#pragma unroll
                for (int e = 0; e < NN; ++e) D[e] = Dm[e * kTile];
                block_inverse<T, NC>(D, inv);
                T *Im = S.Ai + mat_off(L.G, NI, color, t);
#pragma unroll
                for (int e = 0; e < NI; ++e) Im[e * kTile] = inv[e];
            }
        }
        __syncthreads();
    }
    constexpr bool kKeepRegRuns = sizeof(T) == 4;
    RegCell<T, NC> keep[kKeepRegRuns ? 2 : 1];      // unused in FP64
    bool keep_loaded = false;
    for (int q = 0; q < nops; ++q) {
        const CoarseOp op = ops[q];
        const LevelDev &Ld = lv[op.level];
        const LevelDev &Lc = lv[op.level < nl ? op.level + 1 : op.level];
        if (op.kind == COP_RUN) {
            const LdsLevel<T, NC> F(lds, Ld);
            if constexpr (NC == 3) {
                if (op.aux && 4 * Ld.G.plane <= kCoarseBlock) {
                    coarse_run_split<T>(op, Ld.G, F.A, F.Ai, F.b, F.x, zslot);
                    __syncthreads();
                    continue;
                }
            }
            coarse_run<T, NC>(op, Ld.G, F.A, F.Ai, F.b, F.x);
        } else if (op.kind == COP_REGRUN) {
            // FP32: the level's block rows stay in registers from the first
            // run to the end of the program; FP64: reloaded per run (the
            // register file holds them only while no other level's run does)
            coarse_reg_level<T, NC, kKeepRegRuns>(op, Ld, Lc, lds, keep, &keep_loaded);
        } else if (Ld.lds_off >= 0) {
            const LdsLevel<T, NC> F(lds, Ld), Cl(lds, Lc);
            coarse_op<T, NC, true>(op, Ld.G, Lc.G, F.A, F.Ai, F.b, F.x, Cl.b, Cl.x);
        } else if (Lc.lds_off >= 0) {
            const LdsLevel<T, NC> Cl(lds, Lc);
            coarse_op<T, NC, false>(op, Ld.G, Lc.G, in_global((const T *)Ld.A), nullptr,
                                    in_global((const T *)Ld.b), in_global((T *)Ld.x), Cl.b, Cl.x);
        } else {
            coarse_op<T, NC, false>(op, Ld.G, Lc.G, in_global((const T *)Ld.A), nullptr,
                                    in_global((const T *)Ld.b), in_global((T *)Ld.x),
                                    in_global((T *)Lc.b), in_global((const T *)Lc.x));
        }
        __syncthreads();
    }
    if (l_lds >= 0) {
        for (int l = l_lds; l <= nl; ++l) {
            const LevelDev &L = lv[l];
            const LdsLevel<T, NC> S(lds, L);
            const long nv = 2L * NC * L.G.plane;
            T *gb = in_global((T *)L.b), *gx = in_global((T *)L.x);
            for (long k = threadIdx.x; k < nv; k += kCoarseBlock) { gb[k] = S.b[k]; gx[k] = S.x[k]; }
        }
    }
}

// Two consecutive half sweeps of the red-black block Gauss-Seidel smoother
// in one launch, on tiles of kPairTX x kPairTY cells.  Phase 1: colour c in
// MODE for the tile's colour-c cells (one per thread of the first
// kPairCells) and, redundantly, for the kPairRing colour-c cells that border
// the tile (the neighbours of its colour-c^1 cells; one per further thread),
// all kept in LDS; the tile's own go to x.  Phase 2: colour c^1 (normal
// mode) for the tile's cells, reading colour c from LDS; each thread's block
// row is loaded before phase 1 so both phases' loads are in flight together.
// Colour c^1's old values come from xin and its new values go to xout (two
// different buffers: other tiles may still read the old values).  Every
// cell update is sgs_cell's arithmetic on the same inputs, so the result is
// bit for bit that of the two half sweeps launched one by one.
constexpr int kPairCells = kPairTX / 2 * kPairTY;        // cells of one colour per tile
constexpr int kPairRing = kPairTX + kPairTY;             // colour-c cells bordering a tile
constexpr int kPairThreads = (kPairCells + kPairRing + 63) / 64 * 64;

// The pair on the tile with corner (i0, j0) (both even).
template <class T, int NC, int MODE>
__device__ __forceinline__ void sgs_pair_tile(const LevelGeom &G, const T *__restrict__ A,
                                              const T *__restrict__ b, T *__restrict__ x,
                                              const T *__restrict__ xin, T *__restrict__ xout,
                                              int color, const LevelGeom &Gc,
                                              const T *__restrict__ xc, int i0, int j0)
{
    constexpr int NF = 4;
    constexpr int NN = NC * NC;
    constexpr int NE = (NF + 1) * NN;
    constexpr int LX = kPairTX + 2, LY = kPairTY + 2;
    __shared__ T lx[NC][LY][LX];
    const int tid = (int)threadIdx.x;
    const int c1 = color, c2 = color ^ 1;

    // phase 2 cell of this thread and its block row, loaded first
    const bool tile_thread = tid < kPairCells;
    const int j2 = j0 + tid / (kPairTX / 2);
    const int i2 = i0 + 2 * (tid % (kPairTX / 2)) + ((j2 + c2) & 1);
    const bool own2 = tile_thread && i2 < G.nx && j2 < G.ny;
    const long t2 = (long)j2 * G.W + (i2 >> 1);
    T a2[NE], bv2[NC];
    if (own2) {
        const T *Am = A + mat_off(G, NE, c2, t2);
#pragma unroll
        for (int e = 0; e < NE; ++e) a2[e] = Am[e * kTile];
#pragma unroll
        for (int r = 0; r < NC; ++r) bv2[r] = b[((long)c2 * NC + r) * G.plane + t2];
    }

    // phase 1 cell of this thread: a tile cell of colour c, or a bordering one
    int i, j;
    if (tile_thread) {
        j = j0 + tid / (kPairTX / 2);
        i = i0 + 2 * (tid % (kPairTX / 2)) + ((j + c1) & 1);
    } else {
        const int v = tid - kPairCells, h = kPairTY / 2;
        if (v < h) { i = i0 - 1; j = j0 + 2 * v + (c1 ^ 1); }                 // left
        else if (v < 2 * h) { i = i0 + kPairTX; j = j0 + 2 * (v - h) + c1; }  // right
        else if (v < 2 * h + kPairTX / 2) { i = i0 + 2 * (v - 2 * h) + (c1 ^ 1); j = j0 - 1; }
        else { i = i0 + 2 * (v - 2 * h - kPairTX / 2) + c1; j = j0 + kPairTY; }  // top
    }
    const bool own1 = tid < kPairCells + kPairRing && i >= 0 && i < G.nx && j >= 0 && j < G.ny;
    if (own1) {
        const long t = (long)j * G.W + (i >> 1);
        const T *Am = A + mat_off(G, NE, c1, t);
        T a[NE], bv[NC], v[NF][NC], xi[NC];
        bool ok[NF];
#pragma unroll
        for (int e = 0; e < (MODE == MODE_ZERO ? NN : NE); ++e) a[e] = Am[e * kTile];
#pragma unroll
        for (int r = 0; r < NC; ++r) bv[r] = b[((long)c1 * NC + r) * G.plane + t];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            int ni = i, nj = j;
            if (f == FW) { ni = i - 1; ok[f] = i > 0; }
            else if (f == FE) { ni = i + 1; ok[f] = i + 1 < G.nx; }
            else if (f == FS) { nj = j - 1; ok[f] = j > 0; }
            else { nj = j + 1; ok[f] = j + 1 < G.ny; }
            if (MODE != MODE_ZERO) {
                if (ok[f]) {
                    read_other<T, NC, MODE>(G, xin, ni, nj, Gc, xc, v[f]);
                } else {
#pragma unroll
                    for (int q = 0; q < NC; ++q) v[f][q] = T(0);
                }
            }
        }
        gs_update<T, NC, MODE == MODE_ZERO, false>(a, nullptr, bv, v, ok, xi);
#pragma unroll
        for (int r = 0; r < NC; ++r) lx[r][j - j0 + 1][i - i0 + 1] = xi[r];
        if (tile_thread) {
            T *xm = x + (long)c1 * NC * G.plane + t;
#pragma unroll
            for (int r = 0; r < NC; ++r) xm[r * G.plane] = xi[r];
        }
    }
    __syncthreads();

    // phase 2: the tile's colour-c^1 cells, colour c from LDS
    if (!own2) return;
    T v[NF][NC], xi[NC];
    bool ok[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        int ni = i2, nj = j2;
        if (f == FW) { ni = i2 - 1; ok[f] = i2 > 0; }
        else if (f == FE) { ni = i2 + 1; ok[f] = i2 + 1 < G.nx; }
        else if (f == FS) { nj = j2 - 1; ok[f] = j2 > 0; }
        else { nj = j2 + 1; ok[f] = j2 + 1 < G.ny; }
        const int li = ok[f] ? ni - i0 + 1 : 1, lj = ok[f] ? nj - j0 + 1 : 1;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const T val = lx[q][lj][li];
            v[f][q] = ok[f] ? val : T(0);
        }
    }
    gs_update<T, NC, false, false>(a2, nullptr, bv2, v, ok, xi);
#pragma unroll
    for (int r = 0; r < NC; ++r) xout[r * G.plane + t2] = xi[r];
}

template <class T, int NC, int MODE>
__global__ void __launch_bounds__(kPairThreads) k_sgs_pair(LevelGeom G, const T *__restrict__ A,
                                                           const T *__restrict__ b,
                                                           T *__restrict__ x,
                                                           const T *__restrict__ xin,
                                                           T *__restrict__ xout, int color,
                                                           LevelGeom Gc, const T *__restrict__ xc,
                                                           int ntx)
{
    const int tile = xcd_block(blockIdx.x, gridDim.x);
    sgs_pair_tile<T, NC, MODE>(G, A, b, x, xin, xout, color, Gc, xc, (tile % ntx) * kPairTX,
                               (tile / ntx) * kPairTY);
}

// Three consecutive half sweeps (colours c, c^1, c; the first in MODE) in one
// launch, on the tiles of k_sgs_pair: phase 0 updates colour c on the tile
// extended by two cells (neighbours from xin), phase 1 colour c^1 on the tile
// extended by one cell, phase 2 colour c on the tile (neighbours from LDS in
// phases 1 and 2).  Every cell that a later phase reads was computed by the
// previous phase, so each update is sgs_cell's arithmetic on the values the
// separate launches would have produced.  Outputs: colour c^1 of the tile to
// xout (xin is still read by other tiles), colour c to x.  The phase-2 block
// rows are loaded before phase 0.
constexpr int kTripleThreads = ((kPairTX + 4) / 2 * (kPairTY + 4) + 63) / 64 * 64;

template <class T, int NC>
__device__ __forceinline__ void multi_faces(const LevelGeom &G, int i, int j, int *ni, int *nj,
                                            bool *ok)
{
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        ni[f] = i;
        nj[f] = j;
        if (f == FW) { ni[f] = i - 1; ok[f] = i > 0; }
        else if (f == FE) { ni[f] = i + 1; ok[f] = i + 1 < G.nx; }
        else if (f == FS) { nj[f] = j - 1; ok[f] = j > 0; }
        else { nj[f] = j + 1; ok[f] = j + 1 < G.ny; }
    }
}

template <class T, int NC, int MODE>
__global__ void __launch_bounds__(kTripleThreads) k_sgs_triple(LevelGeom G,
                                                               const T *__restrict__ A,
                                                               const T *__restrict__ b,
                                                               T *__restrict__ x,
                                                               const T *__restrict__ xin,
                                                               T *__restrict__ xout, int color,
                                                               LevelGeom Gc,
                                                               const T *__restrict__ xc, int ntx)
{
    constexpr int NF = 4;
    constexpr int NN = NC * NC;
    constexpr int NE = (NF + 1) * NN;
    constexpr int H = 2;
    constexpr int LW = kPairTX + 2 * H, LH = kPairTY + 2 * H;
    __shared__ T lx[NC][LH][LW];
    const int tile = xcd_block(blockIdx.x, gridDim.x);
    const int i0 = (tile % ntx) * kPairTX, j0 = (tile / ntx) * kPairTY;   // both even
    const int tid = (int)threadIdx.x;
    const int c0 = color, c1 = color ^ 1;

    // phase 2 cell (the tile's colour-c cell of this thread), loaded first
    const int j2 = j0 + tid / (kPairTX / 2);
    const int i2 = i0 + 2 * (tid % (kPairTX / 2)) + ((j2 + c0) & 1);
    const bool own2 = tid < kPairCells && i2 < G.nx && j2 < G.ny;
    const long t2 = (long)j2 * G.W + (i2 >> 1);
    T a2[NE], bv2[NC];
    if (own2) {
        const T *Am = A + mat_off(G, NE, c0, t2);
#pragma unroll
        for (int e = 0; e < NE; ++e) a2[e] = Am[e * kTile];
#pragma unroll
        for (int r = 0; r < NC; ++r) bv2[r] = b[((long)c0 * NC + r) * G.plane + t2];
    }

    // phase 0: colour c on the tile extended by 2 (one cell per thread)
    {
        constexpr int WH = (kPairTX + 2 * H) / 2;
        const int jj = j0 - H + tid / WH;
        const int ib = i0 - H;
        const int ii = ib + 2 * (tid % WH) + ((ib + jj + c0) & 1);
        if (tid < WH * (kPairTY + 2 * H) && ii >= 0 && ii < G.nx && jj >= 0 && jj < G.ny) {
            const long t = (long)jj * G.W + (ii >> 1);
            const T *Am = A + mat_off(G, NE, c0, t);
            T a[NE], bv[NC], v[NF][NC], xi[NC];
            int ni[NF], nj[NF];
            bool ok[NF];
            multi_faces<T, NC>(G, ii, jj, ni, nj, ok);
#pragma unroll
            for (int e = 0; e < (MODE == MODE_ZERO ? NN : NE); ++e) a[e] = Am[e * kTile];
#pragma unroll
            for (int r = 0; r < NC; ++r) bv[r] = b[((long)c0 * NC + r) * G.plane + t];
            if (MODE != MODE_ZERO) {
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    if (ok[f]) {
                        read_other<T, NC, MODE>(G, xin, ni[f], nj[f], Gc, xc, v[f]);
                    } else {
#pragma unroll
                        for (int q = 0; q < NC; ++q) v[f][q] = T(0);
                    }
                }
            }
            gs_update<T, NC, MODE == MODE_ZERO, false>(a, nullptr, bv, v, ok, xi);
#pragma unroll
            for (int r = 0; r < NC; ++r) lx[r][jj - j0 + H][ii - i0 + H] = xi[r];
        }
    }
    __syncthreads();

    // phase 1: colour c^1 on the tile extended by 1, neighbours from LDS
    {
        constexpr int WH = (kPairTX + 2) / 2;
        const int jj = j0 - 1 + tid / WH;
        const int ib = i0 - 1;
        const int ii = ib + 2 * (tid % WH) + ((ib + jj + c1) & 1);
        if (tid < WH * (kPairTY + 2) && ii >= 0 && ii < G.nx && jj >= 0 && jj < G.ny) {
            const long t = (long)jj * G.W + (ii >> 1);
            const T *Am = A + mat_off(G, NE, c1, t);
            T a[NE], bv[NC], v[NF][NC], xi[NC];
            int ni[NF], nj[NF];
            bool ok[NF];
            multi_faces<T, NC>(G, ii, jj, ni, nj, ok);
#pragma unroll
            for (int e = 0; e < NE; ++e) a[e] = Am[e * kTile];
#pragma unroll
            for (int r = 0; r < NC; ++r) bv[r] = b[((long)c1 * NC + r) * G.plane + t];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const int li = ok[f] ? ni[f] - i0 + H : H, lj = ok[f] ? nj[f] - j0 + H : H;
#pragma unroll
                for (int q = 0; q < NC; ++q) {
                    const T val = lx[q][lj][li];
                    v[f][q] = ok[f] ? val : T(0);
                }
            }
            gs_update<T, NC, false, false>(a, nullptr, bv, v, ok, xi);
            // colour c^1 slots: no thread reads them in this phase
#pragma unroll
            for (int r = 0; r < NC; ++r) lx[r][jj - j0 + H][ii - i0 + H] = xi[r];
            if (ii >= i0 && ii < i0 + kPairTX && jj >= j0 && jj < j0 + kPairTY) {
#pragma unroll
                for (int r = 0; r < NC; ++r) xout[r * G.plane + t] = xi[r];
            }
        }
    }
    __syncthreads();

    // phase 2: the tile's colour-c cells, neighbours from LDS
    if (!own2) return;
    T v[NF][NC], xi[NC];
    int ni[NF], nj[NF];
    bool ok[NF];
    multi_faces<T, NC>(G, i2, j2, ni, nj, ok);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const int li = ok[f] ? ni[f] - i0 + H : H, lj = ok[f] ? nj[f] - j0 + H : H;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const T val = lx[q][lj][li];
            v[f][q] = ok[f] ? val : T(0);
        }
    }
    gs_update<T, NC, false, false>(a2, nullptr, bv2, v, ok, xi);
    T *xm = x + (long)c0 * NC * G.plane + t2;
#pragma unroll
    for (int r = 0; r < NC; ++r) xm[r * G.plane] = xi[r];
}

// Layout conversions between the public FP64 layouts and the hierarchy's
// colour-split storage of precision T.
template <class T>
__global__ void __launch_bounds__(kBlock) k_to_split(int n, LevelGeom G,
                                                     const double *__restrict__ v,
                                                     T *__restrict__ s)
{
    long idx = (long)blockIdx.x * kBlock + threadIdx.x;
    const long N = (long)G.nx * G.ny;
    if (idx >= N) return;
    int i = (int)(idx % G.nx), j = (int)(idx / G.nx);
    int color = (i + j) & 1;
    T *o = s + (long)color * n * G.plane + (long)j * G.W + (i >> 1);
    for (int c = 0; c < n; ++c) o[c * G.plane] = T(v[c * N + idx]);
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_from_split(int n, LevelGeom G,
                                                       const T *__restrict__ s,
                                                       double *__restrict__ v)
{
    long idx = (long)blockIdx.x * kBlock + threadIdx.x;
    const long N = (long)G.nx * G.ny;
    if (idx >= N) return;
    int i = (int)(idx % G.nx), j = (int)(idx / G.nx);
    int color = (i + j) & 1;
    const T *o = s + (long)color * n * G.plane + (long)j * G.W + (i >> 1);
    for (int c = 0; c < n; ++c) v[c * N + idx] = double(o[c * G.plane]);
}

// Block matrices [NE][ny][nx] (FP64) <-> colour-split tiled layout (T).
template <class T>
__global__ void __launch_bounds__(kBlock) k_mat_to_tiled(int ne, LevelGeom G,
                                                         const double *__restrict__ v,
                                                         T *__restrict__ s)
{
    long idx = (long)blockIdx.x * kBlock + threadIdx.x;
    const long N = (long)G.nx * G.ny;
    if (idx >= N) return;
    int i = (int)(idx % G.nx), j = (int)(idx / G.nx);
    T *o = s + mat_off(G, ne, (i + j) & 1, (long)j * G.W + (i >> 1));
    for (int e = 0; e < ne; ++e) o[e * kTile] = T(v[e * N + idx]);
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_mat_from_tiled(int ne, LevelGeom G,
                                                           const T *__restrict__ s,
                                                           double *__restrict__ v)
{
    long idx = (long)blockIdx.x * kBlock + threadIdx.x;
    const long N = (long)G.nx * G.ny;
    if (idx >= N) return;
    int i = (int)(idx % G.nx), j = (int)(idx / G.nx);
    const T *o = s + mat_off(G, ne, (i + j) & 1, (long)j * G.W + (i >> 1));
    for (int e = 0; e < ne; ++e) v[e * N + idx] = double(o[e * kTile]);
}


// ---------------------------------------------------------------------------
// Sensitivities of the steady state (the adjoint extension).

// Face of the neighbour across face f that faces back.
__device__ __forceinline__ int opposite(int f) { return f ^ 1; }   // W<->E, S<->N

// Block transpose of a level matrix: At's block at slot t (colour c) towards
// neighbour j is A's block at j towards this cell, transposed; the diagonal
// block is transposed in place; blocks pointing out of the grid are zero.
// One thread per slot of both colours.
template <class T, int NC>
__global__ void __launch_bounds__(kBlock) k_transpose(LevelGeom G, const T *__restrict__ A,
                                                      T *__restrict__ At)
{
    constexpr int NF = (NC == 2) ? 2 : 4;
    constexpr int NN = NC * NC;
    constexpr int NE = (NF + 1) * NN;
    const long k = (long)blockIdx.x * kBlock + threadIdx.x;
    if (k >= 2 * G.plane) return;
    const int color = k >= G.plane ? 1 : 0;
    const long t = k - color * G.plane;
    const int j = (int)(t / G.W), kk = (int)(t % G.W);
    const int i = 2 * kk + ((j + color) & 1);
    if (i >= G.nx) return;
    const T *Am = A + mat_off(G, NE, color, t);
    T *Om = At + mat_off(G, NE, color, t);
#pragma unroll
    for (int r = 0; r < NC; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c) Om[(r * NC + c) * kTile] = Am[(c * NC + r) * kTile];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        int ni = i, nj = j;
        bool ok;
        if (f == FW) { ni = i - 1; ok = i > 0; }
        else if (f == FE) { ni = i + 1; ok = i + 1 < G.nx; }
        else if (f == FS) { nj = j - 1; ok = j > 0; }
        else { nj = j + 1; ok = j + 1 < G.ny; }
        if (ok) {
            const T *Nm = A + mat_off(G, NE, color ^ 1, (long)nj * G.W + (ni >> 1)) +
                          (opposite(f) + 1) * NN * kTile;
#pragma unroll
            for (int r = 0; r < NC; ++r)
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    Om[((f + 1) * NN + r * NC + c) * kTile] = Nm[(c * NC + r) * kTile];
        } else {
#pragma unroll
            for (int e = 0; e < NN; ++e) Om[((f + 1) * NN + e) * kTile] = T(0);
        }
    }
}

// Row pins of the Newton matrix applied to one row's bed derivative d.
template <int NC>
__device__ __forceinline__ void pin_bed_row(const Phys &P, const unsigned char *iso,
                                            const double *U, long idx, double *d)
{
    if (iso[idx]) {
#pragma unroll
        for (int r = 0; r < NC; ++r) d[r] = 0.0;
    } else if (P.dry_pin && U[idx] == 0.0) {
#pragma unroll
        for (int r = 1; r < NC; ++r) d[r] = 0.0;
    }
}

// out_j = (dR/dz)^T lam at cell j: the bed of j raised by eps = fd_eps,
// dR_j/dz_j = sum over j's faces (W, E, S, N) of |e| (T(z_j + eps) - T) / eps
// (a boundary face's ghost carries the raised bed), dR_i/dz_j = |e| (T(z_j +
// eps) - T) / eps of each neighbour i's face towards j, rows pinned as in
// the assembly; out_j = lam_j . dR_j/dz_j, then + lam_i . dR_i/dz_j for the
// neighbours in W, E, S, N order, dot products in component order.
template <int NC>
__global__ void __launch_bounds__(kBlock) k_bed_vjp(Phys P, const double *__restrict__ z,
                                                    const double *__restrict__ U,
                                                    const unsigned char *__restrict__ iso,
                                                    const double *__restrict__ lam,
                                                    double *__restrict__ out)
{
    constexpr int NF = (NC == 2) ? 2 : 4;
    const int xb = xcd_block(blockIdx.x, gridDim.x);
    const long idx = (long)xb * kBlock + threadIdx.x;
    const long N = (long)P.nx * P.ny;
    if (idx >= N) return;
    const int i = (int)(idx % P.nx), j = (int)(idx / P.nx);
    const double eps = P.eps;
    double qo[NC];
    load_state<NC>(P, U, idx, qo);
    const Side own = cell_side<NC>(P, qo, z[idx]);
    Side ownp = own;
    ownp.z = z[idx] + eps;
    double d[NC], T0[NC], Tp[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r) d[r] = 0.0;
    for (int f = 0; f < NF; ++f) {
        const double e = P.elen[f];
        int ni, nj;
        if (neighbour(P, i, j, f, ni, nj)) {
            const long nidx = (long)nj * P.nx + ni;
            double qn[NC];
            load_state<NC>(P, U, nidx, qn);
            const Side oth = cell_side<NC>(P, qn, z[nidx]);
            edge_term<NC>(P, f, own, oth, T0);
            edge_term<NC>(P, f, ownp, oth, Tp);
        } else {
            edge_term<NC>(P, f, own, ghost(P, f, own), T0);
            edge_term<NC>(P, f, ownp, ghost(P, f, ownp), Tp);
        }
#pragma unroll
        for (int r = 0; r < NC; ++r) d[r] = d[r] + e * ((Tp[r] - T0[r]) / eps);
    }
    pin_bed_row<NC>(P, iso, U, idx, d);
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < NC; ++r) acc = acc + lam[r * N + idx] * d[r];
    for (int f = 0; f < NF; ++f) {
        int ni, nj;
        if (!neighbour(P, i, j, f, ni, nj)) continue;
        const long nidx = (long)nj * P.nx + ni;
        const int g = opposite(f);
        const double e = P.elen[g];
        double qn[NC];
        load_state<NC>(P, U, nidx, qn);
        const Side nb = cell_side<NC>(P, qn, z[nidx]);
        edge_term<NC>(P, g, nb, own, T0);
        edge_term<NC>(P, g, nb, ownp, Tp);
#pragma unroll
        for (int r = 0; r < NC; ++r) d[r] = e * ((Tp[r] - T0[r]) / eps);
        pin_bed_row<NC>(P, iso, U, nidx, d);
#pragma unroll
        for (int r = 0; r < NC; ++r) acc = acc + lam[r * N + nidx] * d[r];
    }
    out[idx] = acc;
}

// l1 norm of the linear residual b - A x over a level's cells (block sums).
template <class T, int NC>
__global__ void __launch_bounds__(kBlock) k_lin_res_norm(LevelGeom G, const T *__restrict__ A,
                                                         const T *__restrict__ b,
                                                         const T *__restrict__ x,
                                                         double *__restrict__ partial)
{
    const int xb = xcd_block(blockIdx.x, gridDim.x);
    const long idx = (long)xb * kBlock + threadIdx.x;
    double v = 0.0;
    if (idx < (long)G.nx * G.ny) {
        T r[NC];
        lin_residual_cell<T, NC>(G, A, b, x, (int)(idx % G.nx), (int)(idx / G.nx), r);
        v = dabs(double(r[0])) + dabs(double(r[1]));
        if (NC == 3) v = v + dabs(double(r[2]));
    }
    double s = block_sum(v);
    if (threadIdx.x == 0) partial[xb] = s;
}

// Level-0 vector kernels of the Krylov acceleration (FP64 hierarchy,
// colour-split vectors of n = 2 * NC * plane entries).

// y = A x on a level (the linear residual's product: D x_i, then the
// neighbours in W, E, S, N order).
template <int NC>
__global__ void __launch_bounds__(kBlock) k_apply(LevelGeom G, const double *__restrict__ A,
                                                  const double *__restrict__ x,
                                                  double *__restrict__ y)
{
    const int xb = xcd_block(blockIdx.x, gridDim.x);
    const long idx = (long)xb * kBlock + threadIdx.x;
    if (idx >= (long)G.nx * G.ny) return;
    const int i = (int)(idx % G.nx), j = (int)(idx / G.nx);
    double r[NC];
    constexpr int NF = (NC == 2) ? 2 : 4;
    constexpr int NE = (NF + 1) * NC * NC;
    const int color = (i + j) & 1;
    const long slot = (long)j * G.W + (i >> 1);
    const double *Am = A + mat_off(G, NE, color, slot);
    const double *xm = x + (long)color * NC * G.plane + slot;
    const double *xo = x + (long)(color ^ 1) * NC * G.plane;
    double xi[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) xi[c] = xm[c * G.plane];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        r[q] = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) r[q] = r[q] + Am[(q * NC + c) * kTile] * xi[c];
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        int ni = i, nj = j;
        bool ok;
        if (f == FW) { ni = i - 1; ok = i > 0; }
        else if (f == FE) { ni = i + 1; ok = i + 1 < G.nx; }
        else if (f == FS) { nj = j - 1; ok = j > 0; }
        else { nj = j + 1; ok = j + 1 < G.ny; }
        if (!ok) continue;
        const double *pp = xo + (long)nj * G.W + (ni >> 1);
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int c = 0; c < NC; ++c)
                r[q] = r[q] + Am[(((f + 1) * NC + q) * NC + c) * kTile] * pp[c * G.plane];
    }
    double *ym = y + (long)color * NC * G.plane + slot;
#pragma unroll
    for (int q = 0; q < NC; ++q) ym[q * G.plane] = r[q];
}

// r = b - A x as a vector (lin_residual_cell per cell).
template <int NC>
__global__ void __launch_bounds__(kBlock) k_lin_res_vec(LevelGeom G, const double *__restrict__ A,
                                                        const double *__restrict__ b,
                                                        const double *__restrict__ x,
                                                        double *__restrict__ r)
{
    const int xb = xcd_block(blockIdx.x, gridDim.x);
    const long idx = (long)xb * kBlock + threadIdx.x;
    if (idx >= (long)G.nx * G.ny) return;
    const int i = (int)(idx % G.nx), j = (int)(idx / G.nx);
    double v[NC];
    lin_residual_cell<double, NC>(G, A, b, x, i, j, v);
    const int color = (i + j) & 1;
    double *rm = r + (long)color * NC * G.plane + (long)j * G.W + (i >> 1);
#pragma unroll
    for (int q = 0; q < NC; ++q) rm[q * G.plane] = v[q];
}

// partial[k * gridDim.x + block] = sum over the block's entries of
// V_k[e] * w[e], k < nv (vectors V_k = V + k * ld).
__global__ void __launch_bounds__(kBlock) k_multidot(long n, const double *__restrict__ V, long ld,
                                                     int nv, const double *__restrict__ w,
                                                     double *__restrict__ partial)
{
    const long e = (long)blockIdx.x * kBlock + threadIdx.x;
    const double we = e < n ? w[e] : 0.0;
    for (int k = 0; k < nv; ++k) {
        const double v = e < n ? V[k * ld + e] * we : 0.0;
        const double s = block_sum(v);
        if (threadIdx.x == 0) partial[(long)k * gridDim.x + blockIdx.x] = s;
    }
}

// out[k] = sum of partial[k * nparts .. (k + 1) * nparts), one block per k.
__global__ void __launch_bounds__(kBlock) k_multi_reduce(const double *__restrict__ partial,
                                                         int nparts, double *__restrict__ out)
{
    const double *p = partial + (long)blockIdx.x * nparts;
    double v = 0.0;
    for (int q = threadIdx.x; q < nparts; q += kBlock) v = v + p[q];
    const double s = block_sum(v);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// w[e] = a * w[e] - sum over k < nv of c[k] V_k[e] (k in order).
__global__ void __launch_bounds__(kBlock) k_multi_axpy(long n, const double *__restrict__ V, long ld,
                                                       int nv, const double *__restrict__ c,
                                                       double a, double *__restrict__ w)
{
    const long e = (long)blockIdx.x * kBlock + threadIdx.x;
    if (e >= n) return;
    double v = a * w[e];
    for (int k = 0; k < nv; ++k) v = v - c[k] * V[k * ld + e];
    w[e] = v;
}

// ---------------------------------------------------------------------------
// Algorithm 1, Step 1 on the natural layout: child averages onto the next
// coarser mesh, in the child order SW, SE, NW, NE as (((SW + SE) + NW) + NE)
// / 4 (1D: (left + right) / 2), and injection of a coarse state into the
// children.  ncomp component planes of nxf x nyf fine cells.

__global__ void __launch_bounds__(kBlock) k_average(int dim, int nxf, int nyf, int ncomp,
                                                    const double *__restrict__ f,
                                                    double *__restrict__ c)
{
    const int nxc = nxf / 2, nyc = dim == 1 ? 1 : nyf / 2;
    const long Nc = (long)nxc * nyc, Nf = (long)nxf * nyf;
    const long idx = (long)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= Nc) return;
    const int I = (int)(idx % nxc), J = (int)(idx / nxc);
    for (int k = 0; k < ncomp; ++k) {
        const double *q = f + k * Nf;
        double v;
        if (dim == 1) {
            v = (q[2 * I] + q[2 * I + 1]) * 0.5;
        } else {
            const long r0 = (long)2 * J * nxf, r1 = (long)(2 * J + 1) * nxf;
            v = (((q[r0 + 2 * I] + q[r0 + 2 * I + 1]) + q[r1 + 2 * I]) + q[r1 + 2 * I + 1]) * 0.25;
        }
        c[k * Nc + idx] = v;
    }
}

__global__ void __launch_bounds__(kBlock) k_inject(int dim, int nxf, int nyf, int ncomp,
                                                   const double *__restrict__ c,
                                                   double *__restrict__ f)
{
    const int nxc = nxf / 2, nyc = dim == 1 ? 1 : nyf / 2;
    const long Nc = (long)nxc * nyc, Nf = (long)nxf * nyf;
    const long idx = (long)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= Nf) return;
    const int i = (int)(idx % nxf), j = (int)(idx / nxf);
    const long src = (long)(dim == 1 ? 0 : j / 2) * nxc + i / 2;
    for (int k = 0; k < ncomp; ++k) f[k * Nf + idx] = c[k * Nc + src];
}

// ---------------------------------------------------------------------------
// Batched kernels: one block per work item (instance, tile), in XCD-aware
// order; the per-cell work is the same function as in the single-problem
// kernels, so every instance's results are those of its own solve.  Tiles of
// the reduction kernels are the 256-cell blocks of the single kernels, and an
// instance's tiles are contiguous in the work list, so its partial sums are
// the single kernel's partial sums.

__device__ __forceinline__ WorkItem work_item(const WorkRange &w, int &pos)
{
    pos = xcd_block(blockIdx.x, gridDim.x);
    return w.items[pos];
}

template <int NC>
__global__ void __launch_bounds__(kBlock) kb_isolated(const BatchInst *__restrict__ bi,
                                                      WorkRange w, const int *__restrict__ active)
{
    int pos;
    const WorkItem it = work_item(w, pos);
    if (!active[it.inst]) return;
    const BatchInst &I = bi[it.inst];
    const long idx = (long)it.tile * kBlock + threadIdx.x;
    if (idx < (long)I.P.nx * I.P.ny) isolated_cell<NC>(I.P, in_global(I.z), in_global(I.U), in_global(I.iso), idx);
}

template <int NC, class T>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) kb_assemble(const BatchInst *__restrict__ bi,
                                                      WorkRange w, const int *__restrict__ active,
                                                      double *__restrict__ partial)
{
    int pos;
    const WorkItem it = work_item(w, pos);
    if (!active[it.inst]) return;
    const BatchInst &I = bi[it.inst];
    const long idx = (long)it.tile * kBlock + threadIdx.x;
    double nrm = 0.0;
    if (idx < (long)I.P.nx * I.P.ny)
        nrm = assemble_cell<NC, T>(I.P, I.G0, in_global(I.z), in_global(I.U), in_global(I.iso),
                                  in_global((T *)I.A), in_global((T *)I.b), nullptr, idx);
    double s = block_sum(nrm);
    if (threadIdx.x == 0) partial[pos] = s;
}

template <int NC>
__global__ void __launch_bounds__(kBlock) kb_residual(const BatchInst *__restrict__ bi,
                                                      WorkRange w, const int *__restrict__ active,
                                                      double *__restrict__ partial)
{
    int pos;
    const WorkItem it = work_item(w, pos);
    if (!active[it.inst]) return;
    const BatchInst &I = bi[it.inst];
    const long idx = (long)it.tile * kBlock + threadIdx.x;
    double nrm = 0.0;
    if (idx < (long)I.P.nx * I.P.ny) nrm = residual_cell<NC>(I.P, in_global(I.z), in_global(I.U), nullptr, idx);
    double s = block_sum(nrm);
    if (threadIdx.x == 0) partial[pos] = s;
}

__global__ void __launch_bounds__(kBlock) kb_count_iso(const BatchInst *__restrict__ bi,
                                                       WorkRange w,
                                                       const int *__restrict__ active,
                                                       double *__restrict__ partial)
{
    int pos;
    const WorkItem it = work_item(w, pos);
    if (!active[it.inst]) return;
    const BatchInst &I = bi[it.inst];
    const long idx = (long)it.tile * kBlock + threadIdx.x;
    double c = (idx < (long)I.P.nx * I.P.ny && in_global(I.iso)[idx]) ? 1.0 : 0.0;
    double s = block_sum(c);
    if (threadIdx.x == 0) partial[pos] = s;
}

__global__ void __launch_bounds__(kBlock) kb_reduce(const double *__restrict__ partial,
                                                    const int *__restrict__ off,
                                                    const int *__restrict__ cnt,
                                                    const int *__restrict__ active,
                                                    double *__restrict__ out)
{
    const int k = blockIdx.x;
    if (!active[k]) return;
    const double *p = partial + off[k];
    const int n = cnt[k];
    double v = 0.0;
    for (int q = threadIdx.x; q < n; q += kBlock) v = v + p[q];
    double s = block_sum(v);
    if (threadIdx.x == 0) out[k] = s;
}

template <int NC>
__global__ void __launch_bounds__(kBlock) kb_blu_half(const BatchInst *__restrict__ bi,
                                                      WorkRange w, const int *__restrict__ active,
                                                      int color)
{
    int pos;
    const WorkItem it = work_item(w, pos);
    if (!active[it.inst]) return;
    const BatchInst &I = bi[it.inst];
    const long t = (long)it.tile * kBlock + threadIdx.x;
    if (t < I.G0.plane) blu_cell<NC>(I.P, in_global(I.z), in_global(I.U), color, t);
}

template <int NC, class T>
__global__ void __launch_bounds__(kBlock) kb_update(const BatchInst *__restrict__ bi,
                                                    WorkRange w, const int *__restrict__ active)
{
    int pos;
    const WorkItem it = work_item(w, pos);
    if (!active[it.inst]) return;
    const BatchInst &I = bi[it.inst];
    const long idx = (long)it.tile * kBlock + threadIdx.x;
    if (idx < (long)I.P.nx * I.P.ny) update_cell<NC, T>(I.P, I.G0, in_global((const T *)I.x), in_global(I.U), idx);
}

template <int NC>
__global__ void __launch_bounds__(kBlock) kb_threshold(const BatchInst *__restrict__ bi,
                                                       WorkRange w,
                                                       const int *__restrict__ active)
{
    int pos;
    const WorkItem it = work_item(w, pos);
    if (!active[it.inst]) return;
    const BatchInst &I = bi[it.inst];
    const long idx = (long)it.tile * kBlock + threadIdx.x;
    if (idx < (long)I.P.nx * I.P.ny) threshold_cell<NC>(I.P, in_global(I.U), idx);
}

template <int NC>
__global__ void __launch_bounds__(kBlock) kb_copy_state(const BatchInst *__restrict__ bi,
                                                        WorkRange w,
                                                        const int *__restrict__ active, int dir)
{
    int pos;
    const WorkItem it = work_item(w, pos);
    if (!active[it.inst]) return;
    const BatchInst &I = bi[it.inst];
    const long N = (long)I.P.nx * I.P.ny;
    const long idx = (long)it.tile * kBlock + threadIdx.x;
    if (idx >= N) return;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double *U = in_global(I.U), *Ulast = in_global(I.Ulast);
        if (dir == 0)
            Ulast[c * N + idx] = U[c * N + idx];
        else
            U[c * N + idx] = Ulast[c * N + idx];
    }
}

template <class T, int NC, int MODE, int TB>
__global__ void __launch_bounds__(TB) kb_sgs_half(const BatchLevel *__restrict__ lv, WorkRange w,
                                                  const int *__restrict__ active, int color)
{
    int pos;
    const WorkItem it = work_item(w, pos);
    if (!active[it.inst]) return;
    const BatchLevel L = global_view(lv[it.inst]);
    const long t = (long)it.tile * TB + threadIdx.x;
    if (t < L.G.plane)
        sgs_cell<T, NC, MODE>(L.G, (const T *)L.A, nullptr, (const T *)L.b, (T *)L.x, color, L.Gc,
                              (const T *)L.xc, t);
}

// kb_sgs_half as a persistent kernel: a fixed grid whose blocks loop over
// the work list (block b takes items b, b + gridDim.x, ...).
template <class T, int NC, int MODE, int TB>
__global__ void __launch_bounds__(TB) kb_sgs_half_loop(const BatchLevel *__restrict__ lv,
                                                       WorkRange w,
                                                       const int *__restrict__ active, int color)
{
    for (int pos = blockIdx.x; pos < w.n; pos += gridDim.x) {
        const WorkItem it = w.items[pos];
        if (!active[it.inst]) continue;
        const BatchLevel L = global_view(lv[it.inst]);
        const long t = (long)it.tile * TB + threadIdx.x;
        if (t < L.G.plane)
            sgs_cell<T, NC, MODE>(L.G, (const T *)L.A, nullptr, (const T *)L.b, (T *)L.x, color,
                                  L.Gc, (const T *)L.xc, t);
    }
}

template <class T, int NC, int TB>
__global__ void __launch_bounds__(TB) kb_sgs_half_res(const BatchLevel *__restrict__ lv,
                                                      WorkRange w, const int *__restrict__ active,
                                                      int color)
{
    int pos;
    const WorkItem it = work_item(w, pos);
    if (!active[it.inst]) return;
    const BatchLevel L = global_view(lv[it.inst]);
    const long t = (long)it.tile * TB + threadIdx.x;
    if (t < L.G.plane)
        sgs_cell<T, NC, MODE_NORMAL, false, false, true>(L.G, (const T *)L.A, nullptr,
                                                         (const T *)L.b, (T *)L.x, color, L.G,
                                                         nullptr, t, (T *)L.rr);
}

template <class T, int MODE>
__global__ void __launch_bounds__(kPairThreads) kb_sgs_pair(const BatchLevel *__restrict__ lv,
                                                            WorkRange w,
                                                            const int *__restrict__ active,
                                                            int color, int flip)
{
    int pos;
    const WorkItem it = work_item(w, pos);
    if (!active[it.inst]) return;
    const BatchLevel L = global_view(lv[it.inst]);
    const int ntx = (L.G.nx + kPairTX - 1) / kPairTX;
    T *x2 = (T *)L.x + (long)(color ^ 1) * 3 * L.G.plane;
    const T *xin = flip ? (const T *)L.xt : x2;
    T *xout = flip ? x2 : (T *)L.xt;
    sgs_pair_tile<T, 3, MODE>(L.G, (const T *)L.A, (const T *)L.b, (T *)L.x, xin, xout, color,
                              L.Gc, (const T *)L.xc, (it.tile % ntx) * kPairTX,
                              (it.tile / ntx) * kPairTY);
}

template <class T, int NC>
__global__ void __launch_bounds__(kBlock) kb_restrict(const BatchLevel *__restrict__ lv,
                                                      WorkRange w,
                                                      const int *__restrict__ active)
{
    int pos;
    const WorkItem it = work_item(w, pos);
    if (!active[it.inst]) return;
    const BatchLevel L = global_view(lv[it.inst]);
    // tiles of kBlock children = kBlock / nch coarse cells
    restrict_block<T, NC>(L.G, (const T *)L.A, (const T *)L.b, (const T *)L.x, L.Gc, (T *)L.bc,
                          (long)it.tile * (kBlock / ((NC == 2) ? 2 : 4)));
}

template <class T, int NC>
__global__ void __launch_bounds__(kBlock) kb_restrict_res(const BatchLevel *__restrict__ lv,
                                                          WorkRange w,
                                                          const int *__restrict__ active, int rcol)
{
    int pos;
    const WorkItem it = work_item(w, pos);
    if (!active[it.inst]) return;
    const BatchLevel L = global_view(lv[it.inst]);
    restrict_block<T, NC, false, true>(L.G, (const T *)L.A, (const T *)L.b, (const T *)L.x, L.Gc,
                                       (T *)L.bc, (long)it.tile * (kBlock / ((NC == 2) ? 2 : 4)),
                                       (const T *)L.rr, rcol);
}

template <class T, int NC>
__global__ void __launch_bounds__(kBlock) kb_fix_color(const BatchLevel *__restrict__ lv,
                                                       WorkRange w,
                                                       const int *__restrict__ active, int op,
                                                       int color)
{
    int pos;
    const WorkItem it = work_item(w, pos);
    if (!active[it.inst]) return;
    const BatchLevel L = global_view(lv[it.inst]);
    const long t = (long)it.tile * kBlock + threadIdx.x;
    if (t < L.G.plane) fix_cell<T, NC>(L.G, op, (T *)L.x, color, L.Gc, (const T *)L.xc, t);
}

template <class T, int NC>
__global__ void __launch_bounds__(kBlock) kb_galerkin(const BatchLevel *__restrict__ lv,
                                                      WorkRange w,
                                                      const int *__restrict__ active)
{
    int pos;
    const WorkItem it = work_item(w, pos);
    if (!active[it.inst]) return;
    const BatchLevel L = global_view(lv[it.inst]);
    const long t = (long)it.tile * kBlock + threadIdx.x;
    if (t < (long)L.Gc.nx * L.Gc.ny) galerkin_cell<T, NC>(L.G, (const T *)L.A, L.Gc, (T *)L.Ac, t);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.

#define NMG_LAUNCH(kern, grid, ...)                                                   \
    do {                                                                              \
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, __VA_ARGS__);        \
        return hipGetLastError();                                                     \
    } while (0)

hipError_t launch_isolated(const Phys &P, const double *z, const double *U, unsigned char *iso,
                           hipStream_t s)
{
    int g = nblocks((long)P.nx * P.ny);
    if (P.dim == 1) NMG_LAUNCH(k_isolated<2>, g, P, z, U, iso);
    NMG_LAUNCH(k_isolated<3>, g, P, z, U, iso);
}

hipError_t launch_assemble(const Phys &P, const LevelGeom &G, const double *z, const double *U,
                           const unsigned char *iso, void *A, void *b, bool f32, double *R_out,
                           double *partial, hipStream_t s)
{
    int g = nblocks((long)P.nx * P.ny);
    if (f32) {
        if (P.dim == 1)
            NMG_LAUNCH((k_assemble<2, float>), g, P, G, z, U, iso, (float *)A, (float *)b, R_out, partial);
        NMG_LAUNCH((k_assemble<3, float>), g, P, G, z, U, iso, (float *)A, (float *)b, R_out, partial);
    }
    if (P.dim == 1)
        NMG_LAUNCH((k_assemble<2, double>), g, P, G, z, U, iso, (double *)A, (double *)b, R_out, partial);
    NMG_LAUNCH((k_assemble<3, double>), g, P, G, z, U, iso, (double *)A, (double *)b, R_out, partial);
}

hipError_t launch_residual(const Phys &P, const double *z, const double *U, double *R_out,
                           double *partial, hipStream_t s)
{
    int g = nblocks((long)P.nx * P.ny);
    if (P.dim == 1) NMG_LAUNCH(k_residual<2>, g, P, z, U, R_out, partial);
    NMG_LAUNCH(k_residual<3>, g, P, z, U, R_out, partial);
}

hipError_t launch_step1_reset(int *ctrl, hipStream_t s)
{
    hipLaunchKernelGGL(k_step1_reset, dim3(1), dim3(1), 0, s, ctrl);
    return hipGetLastError();
}

hipError_t launch_reduce(const double *partial, int n, double *out, hipStream_t s)
{
    NMG_LAUNCH(k_reduce, 1, partial, n, out);
}

hipError_t launch_count_u8(const unsigned char *v, long n, double *partial, hipStream_t s)
{
    NMG_LAUNCH(k_count_u8, nblocks(n), v, n, partial);
}

// Lanes per cell of a BLU-SGS half sweep: the requested count (1, 4 or 16;
// 16 is 4 in 1D), or by the mesh when negative.
static int blu_lanes(const Phys &P, int lanes)
{
    const long cells = (long)((P.nx + 1) / 2) * P.ny;
    if (lanes < 0) lanes = (cells <= kBluX16MaxCells) ? 16 : (cells <= kBluQuadMaxCells) ? 4 : 1;
    if (lanes >= 16) return P.dim == 2 ? 16 : 4;
    return lanes >= 4 ? 4 : 1;
}

int blu_half_blocks(const Phys &P, int lanes)
{
    const long cells = (long)((P.nx + 1) / 2) * P.ny;
    return nblocks(blu_lanes(P, lanes) * cells);
}

hipError_t launch_blu_half_io(const Phys &P, const double *z, const double *Uown,
                              const double *Unb, double *Uout, int color, int reps, int lanes,
                              hipStream_t s, const int *gate, const StopTest &test,
                              double *res_partial)
{
    if (reps < 1) return hipSuccess;
    lanes = blu_lanes(P, lanes);
    const int g = blu_half_blocks(P, lanes);
    if (lanes == 16)
        NMG_LAUNCH(k_blu_half_x16, g, P, z, Uown, Unb, Uout, color, reps, gate, test, res_partial);
    if (lanes == 4) {
        if (P.dim == 1)
            NMG_LAUNCH(k_blu_half_quad<2>, g, P, z, Uown, Unb, Uout, color, reps, gate, test,
                       res_partial);
        NMG_LAUNCH(k_blu_half_quad<3>, g, P, z, Uown, Unb, Uout, color, reps, gate, test,
                   res_partial);
    }
    if (P.dim == 1)
        NMG_LAUNCH(k_blu_half<2>, g, P, z, Uown, Unb, Uout, color, reps, gate, test, res_partial);
    NMG_LAUNCH(k_blu_half<3>, g, P, z, Uown, Unb, Uout, color, reps, gate, test, res_partial);
}

hipError_t launch_blu_half(const Phys &P, const double *z, double *U, int color, int reps,
                           int lanes, hipStream_t s, const int *gate, const StopTest &test)
{
    return launch_blu_half_io(P, z, U, U, U, color, reps, lanes, s, gate, test, nullptr);
}

hipError_t launch_blu_sweeps(const Phys &P, const double *z, double *U, int n, int lanes,
                             hipStream_t s, const int *gate, const StopTest &test)
{
    const int order[4] = {0, 1, 1, 0};
    int color = -1, reps = 0, launched = 0;
    for (int h = 0; h <= 4 * n; ++h) {
        const int c = (h < 4 * n) ? order[h & 3] : -1;
        if (c == color) {
            ++reps;
            continue;
        }
        if (reps > 0) {
            hipError_t e = launch_blu_half(P, z, U, color, reps, lanes, s, gate,
                                           launched == 0 ? test : StopTest());
            if (e != hipSuccess) return e;
            ++launched;
        }
        color = c;
        reps = 1;
    }
    return hipSuccess;
}

hipError_t launch_update(const Phys &P, const LevelGeom &G, const void *x, bool f32, double *U,
                         hipStream_t s)
{
    int g = nblocks((long)P.nx * P.ny);
    if (f32) {
        if (P.dim == 1) NMG_LAUNCH((k_update<2, float>), g, P, G, (const float *)x, U);
        NMG_LAUNCH((k_update<3, float>), g, P, G, (const float *)x, U);
    }
    if (P.dim == 1) NMG_LAUNCH((k_update<2, double>), g, P, G, (const double *)x, U);
    NMG_LAUNCH((k_update<3, double>), g, P, G, (const double *)x, U);
}

hipError_t launch_threshold(const Phys &P, double *U, hipStream_t s)
{
    int g = nblocks((long)P.nx * P.ny);
    if (P.dim == 1) NMG_LAUNCH(k_threshold<2>, g, P, U);
    NMG_LAUNCH(k_threshold<3>, g, P, U);
}

template <class T, int NC, bool ST>
static hipError_t sgs_dispatch(int mode, const LevelGeom &G, const T *A, const T *b, T *x,
                               int color, const LevelGeom &Gc, const T *xc, hipStream_t s)
{
    int g = nblocks(G.plane);
    switch (mode) {
    case MODE_NORMAL: NMG_LAUNCH((k_sgs_half<T, NC, MODE_NORMAL, ST>), g, G, A, b, x, color, Gc, xc);
    case MODE_ZERO: NMG_LAUNCH((k_sgs_half<T, NC, MODE_ZERO, ST>), g, G, A, b, x, color, Gc, xc);
    case MODE_PROLONG: NMG_LAUNCH((k_sgs_half<T, NC, MODE_PROLONG, ST>), g, G, A, b, x, color, Gc, xc);
    default: NMG_LAUNCH((k_sgs_half<T, NC, MODE_PROLONG_ZERO, ST>), g, G, A, b, x, color, Gc, xc);
    }
}

template <class T, int NC>
static hipError_t sgs_stream(bool stream, int mode, const LevelGeom &G, const void *A,
                             const void *b, void *x, int color, const LevelGeom &Gc,
                             const void *xc, hipStream_t s)
{
    if (stream)
        return sgs_dispatch<T, NC, true>(mode, G, (const T *)A, (const T *)b, (T *)x, color, Gc,
                                         (const T *)xc, s);
    return sgs_dispatch<T, NC, false>(mode, G, (const T *)A, (const T *)b, (T *)x, color, Gc,
                                      (const T *)xc, s);
}

hipError_t launch_sgs_half(int dim, bool f32, int mode, const LevelGeom &G, const void *A,
                           const void *b, void *x, int color, const LevelGeom &Gc, const void *xc,
                           bool stream, hipStream_t s)
{
    if (f32) {
        if (dim == 1) return sgs_stream<float, 2>(stream, mode, G, A, b, x, color, Gc, xc, s);
        return sgs_stream<float, 3>(stream, mode, G, A, b, x, color, Gc, xc, s);
    }
    if (dim == 1) return sgs_stream<double, 2>(stream, mode, G, A, b, x, color, Gc, xc, s);
    return sgs_stream<double, 3>(stream, mode, G, A, b, x, color, Gc, xc, s);
}

template <class T, int NC>
static hipError_t sgs_res_stream(bool stream, const LevelGeom &G, const void *A, const void *b,
                                 void *x, int color, void *rout, hipStream_t s)
{
    int g = nblocks(G.plane);
    if (stream)
        NMG_LAUNCH((k_sgs_half_res<T, NC, true>), g, G, (const T *)A, (const T *)b, (T *)x, color,
                   (T *)rout);
    NMG_LAUNCH((k_sgs_half_res<T, NC, false>), g, G, (const T *)A, (const T *)b, (T *)x, color,
               (T *)rout);
}

hipError_t launch_sgs_half_res(int dim, bool f32, const LevelGeom &G, const void *A,
                               const void *b, void *x, int color, void *rout, bool stream,
                               hipStream_t s)
{
    if (f32) {
        if (dim == 1) return sgs_res_stream<float, 2>(stream, G, A, b, x, color, rout, s);
        return sgs_res_stream<float, 3>(stream, G, A, b, x, color, rout, s);
    }
    if (dim == 1) return sgs_res_stream<double, 2>(stream, G, A, b, x, color, rout, s);
    return sgs_res_stream<double, 3>(stream, G, A, b, x, color, rout, s);
}

template <class T>
static hipError_t pair_dispatch(int mode, const LevelGeom &G, const T *A, const T *b, T *x,
                                const T *xin, T *xout, int color, const LevelGeom &Gc, const T *xc,
                                hipStream_t s)
{
    const int ntx = (G.nx + kPairTX - 1) / kPairTX, nty = (G.ny + kPairTY - 1) / kPairTY;
    const int g = ntx * nty;
#define NMG_PAIR(M)                                                                           \
    do {                                                                                      \
        hipLaunchKernelGGL((k_sgs_pair<T, 3, M>), dim3(g), dim3(kPairThreads), 0, s, G, A, b, \
                           x, xin, xout, color, Gc, xc, ntx);                                 \
        return hipGetLastError();                                                             \
    } while (0)
    switch (mode) {
    case MODE_NORMAL: NMG_PAIR(MODE_NORMAL);
    case MODE_ZERO: NMG_PAIR(MODE_ZERO);
    case MODE_PROLONG: NMG_PAIR(MODE_PROLONG);
    default: NMG_PAIR(MODE_PROLONG_ZERO);
    }
#undef NMG_PAIR
}

hipError_t launch_sgs_pair(bool f32, int mode, const LevelGeom &G, const void *A, const void *b,
                           void *x, const void *xin, void *xout, int color, const LevelGeom &Gc,
                           const void *xc, hipStream_t s)
{
    if (f32)
        return pair_dispatch<float>(mode, G, (const float *)A, (const float *)b, (float *)x,
                                    (const float *)xin, (float *)xout, color, Gc,
                                    (const float *)xc, s);
    return pair_dispatch<double>(mode, G, (const double *)A, (const double *)b, (double *)x,
                                 (const double *)xin, (double *)xout, color, Gc,
                                 (const double *)xc, s);
}

template <class T>
static hipError_t triple_dispatch(int mode, const LevelGeom &G, const T *A, const T *b, T *x,
                                  const T *xin, T *xout, int color, const LevelGeom &Gc,
                                  const T *xc, hipStream_t s)
{
    const int ntx = (G.nx + kPairTX - 1) / kPairTX, nty = (G.ny + kPairTY - 1) / kPairTY;
    const int g = ntx * nty;
#define NMG_TRIPLE(M)                                                                         \
    do {                                                                                      \
        hipLaunchKernelGGL((k_sgs_triple<T, 3, M>), dim3(g), dim3(kTripleThreads), 0, s, G,   \
                           A, b, x, xin, xout, color, Gc, xc, ntx);                           \
        return hipGetLastError();                                                             \
    } while (0)
    switch (mode) {
    case MODE_NORMAL: NMG_TRIPLE(MODE_NORMAL);
    case MODE_ZERO: NMG_TRIPLE(MODE_ZERO);
    case MODE_PROLONG: NMG_TRIPLE(MODE_PROLONG);
    default: NMG_TRIPLE(MODE_PROLONG_ZERO);
    }
#undef NMG_TRIPLE
}

hipError_t launch_sgs_triple(bool f32, int mode, const LevelGeom &G, const void *A,
                             const void *b, void *x, const void *xin, void *xout, int color,
                             const LevelGeom &Gc, const void *xc, hipStream_t s)
{
    if (f32)
        return triple_dispatch<float>(mode, G, (const float *)A, (const float *)b, (float *)x,
                                      (const float *)xin, (float *)xout, color, Gc,
                                      (const float *)xc, s);
    return triple_dispatch<double>(mode, G, (const double *)A, (const double *)b, (double *)x,
                                   (const double *)xin, (double *)xout, color, Gc,
                                   (const double *)xc, s);
}

template <class T, int NC>
static hipError_t restrict_stream(bool stream, const LevelGeom &G, const void *A, const void *b,
                                  const void *x, const LevelGeom &Gc, void *bc, hipStream_t s)
{
    int g = nblocks((long)Gc.nx * Gc.ny * (NC == 2 ? 2 : 4));
    if (stream)
        NMG_LAUNCH((k_restrict<T, NC, true>), g, G, (const T *)A, (const T *)b, (const T *)x, Gc,
                   (T *)bc);
    NMG_LAUNCH((k_restrict<T, NC, false>), g, G, (const T *)A, (const T *)b, (const T *)x, Gc,
               (T *)bc);
}

hipError_t launch_restrict(int dim, bool f32, const LevelGeom &G, const void *A, const void *b,
                           const void *x, const LevelGeom &Gc, void *bc, bool stream,
                           hipStream_t s)
{
    if (f32) {
        if (dim == 1) return restrict_stream<float, 2>(stream, G, A, b, x, Gc, bc, s);
        return restrict_stream<float, 3>(stream, G, A, b, x, Gc, bc, s);
    }
    if (dim == 1) return restrict_stream<double, 2>(stream, G, A, b, x, Gc, bc, s);
    return restrict_stream<double, 3>(stream, G, A, b, x, Gc, bc, s);
}

template <class T, int NC>
static hipError_t restrict_res_stream(bool stream, const LevelGeom &G, const void *A,
                                      const void *b, const void *x, const LevelGeom &Gc, void *bc,
                                      const void *rin, int rcol, hipStream_t s)
{
    int g = nblocks((long)Gc.nx * Gc.ny * (NC == 2 ? 2 : 4));
    if (stream)
        NMG_LAUNCH((k_restrict_res<T, NC, true>), g, G, (const T *)A, (const T *)b, (const T *)x,
                   Gc, (T *)bc, (const T *)rin, rcol);
    NMG_LAUNCH((k_restrict_res<T, NC, false>), g, G, (const T *)A, (const T *)b, (const T *)x, Gc,
               (T *)bc, (const T *)rin, rcol);
}

hipError_t launch_restrict_res(int dim, bool f32, const LevelGeom &G, const void *A,
                               const void *b, const void *x, const LevelGeom &Gc, void *bc,
                               const void *rin, int rcol, bool stream, hipStream_t s)
{
    if (f32) {
        if (dim == 1) return restrict_res_stream<float, 2>(stream, G, A, b, x, Gc, bc, rin, rcol, s);
        return restrict_res_stream<float, 3>(stream, G, A, b, x, Gc, bc, rin, rcol, s);
    }
    if (dim == 1) return restrict_res_stream<double, 2>(stream, G, A, b, x, Gc, bc, rin, rcol, s);
    return restrict_res_stream<double, 3>(stream, G, A, b, x, Gc, bc, rin, rcol, s);
}

hipError_t launch_galerkin(int dim, bool f32, const LevelGeom &Gf, const void *Af,
                           const LevelGeom &Gc, void *Ac, hipStream_t s)
{
    int g = nblocks((long)Gc.nx * Gc.ny);
    if (f32) {
        if (dim == 1) NMG_LAUNCH((k_galerkin<float, 2>), g, Gf, (const float *)Af, Gc, (float *)Ac);
        if (Gf.planeP * 45L * 2 * 4 > (64L << 20))
            NMG_LAUNCH((k_galerkin<float, 3, true>), g, Gf, (const float *)Af, Gc, (float *)Ac);
        NMG_LAUNCH((k_galerkin<float, 3>), g, Gf, (const float *)Af, Gc, (float *)Ac);
    }
    if (dim == 1) NMG_LAUNCH((k_galerkin<double, 2>), g, Gf, (const double *)Af, Gc, (double *)Ac);
    // the finest level's blocks stream through once: non-temporal loads
    if (Gf.planeP * 45L * 2 * 8 > (64L << 20))
        NMG_LAUNCH((k_galerkin<double, 3, true>), g, Gf, (const double *)Af, Gc, (double *)Ac);
    NMG_LAUNCH((k_galerkin<double, 3>), g, Gf, (const double *)Af, Gc, (double *)Ac);
}

hipError_t launch_fix_color(int dim, bool f32, int op, const LevelGeom &G, void *x, int color,
                            const LevelGeom &Gc, const void *xc, hipStream_t s)
{
    int g = nblocks(G.plane);
    if (f32) {
        if (dim == 1) NMG_LAUNCH((k_fix_color<float, 2>), g, G, op, (float *)x, color, Gc, (const float *)xc);
        NMG_LAUNCH((k_fix_color<float, 3>), g, G, op, (float *)x, color, Gc, (const float *)xc);
    }
    if (dim == 1) NMG_LAUNCH((k_fix_color<double, 2>), g, G, op, (double *)x, color, Gc, (const double *)xc);
    NMG_LAUNCH((k_fix_color<double, 3>), g, G, op, (double *)x, color, Gc, (const double *)xc);
}

hipError_t launch_coarse_cycle(int dim, bool f32, const CoarseOp *ops, int nops,
                               const LevelDev *lv, int l_lds, int nl, hipStream_t s)
{
#define NMG_COARSE(T, NC)                                                                     \
    do {                                                                                      \
        hipLaunchKernelGGL((k_coarse_cycle<T, NC>), dim3(1), dim3(kCoarseBlock), 0, s, ops,   \
                           nops, lv, nullptr, l_lds, nl);                                     \
        return hipGetLastError();                                                             \
    } while (0)
    if (f32) {
        if (dim == 1) NMG_COARSE(float, 2);
        NMG_COARSE(float, 3);
    }
    if (dim == 1) NMG_COARSE(double, 2);
    NMG_COARSE(double, 3);
#undef NMG_COARSE
}


// ---- sensitivities ----

hipError_t launch_transpose(int dim, bool f32, const LevelGeom &G, const void *A, void *At,
                            hipStream_t s)
{
    int g = nblocks(2 * G.plane);
    if (f32) {
        if (dim == 1) NMG_LAUNCH((k_transpose<float, 2>), g, G, (const float *)A, (float *)At);
        NMG_LAUNCH((k_transpose<float, 3>), g, G, (const float *)A, (float *)At);
    }
    if (dim == 1) NMG_LAUNCH((k_transpose<double, 2>), g, G, (const double *)A, (double *)At);
    NMG_LAUNCH((k_transpose<double, 3>), g, G, (const double *)A, (double *)At);
}

hipError_t launch_bed_vjp(const Phys &P, const double *z, const double *U,
                          const unsigned char *iso, const double *lam, double *out, hipStream_t s)
{
    int g = nblocks((long)P.nx * P.ny);
    if (P.dim == 1) NMG_LAUNCH(k_bed_vjp<2>, g, P, z, U, iso, lam, out);
    NMG_LAUNCH(k_bed_vjp<3>, g, P, z, U, iso, lam, out);
}

hipError_t launch_lin_res_norm(int dim, bool f32, const LevelGeom &G, const void *A,
                               const void *b, const void *x, double *partial, hipStream_t s)
{
    int g = nblocks((long)G.nx * G.ny);
    if (f32) {
        if (dim == 1) NMG_LAUNCH((k_lin_res_norm<float, 2>), g, G, (const float *)A, (const float *)b, (const float *)x, partial);
        NMG_LAUNCH((k_lin_res_norm<float, 3>), g, G, (const float *)A, (const float *)b, (const float *)x, partial);
    }
    if (dim == 1) NMG_LAUNCH((k_lin_res_norm<double, 2>), g, G, (const double *)A, (const double *)b, (const double *)x, partial);
    NMG_LAUNCH((k_lin_res_norm<double, 3>), g, G, (const double *)A, (const double *)b, (const double *)x, partial);
}

hipError_t launch_apply(int dim, const LevelGeom &G, const double *A, const double *x, double *y,
                        hipStream_t s)
{
    int g = nblocks((long)G.nx * G.ny);
    if (dim == 1) NMG_LAUNCH(k_apply<2>, g, G, A, x, y);
    NMG_LAUNCH(k_apply<3>, g, G, A, x, y);
}

hipError_t launch_lin_res_vec(int dim, const LevelGeom &G, const double *A, const double *b,
                              const double *x, double *r, hipStream_t s)
{
    int g = nblocks((long)G.nx * G.ny);
    if (dim == 1) NMG_LAUNCH(k_lin_res_vec<2>, g, G, A, b, x, r);
    NMG_LAUNCH(k_lin_res_vec<3>, g, G, A, b, x, r);
}

hipError_t launch_multidot(long n, const double *V, long ld, int nv, const double *w,
                           double *partial, double *out, hipStream_t s)
{
    if (nv <= 0) return hipSuccess;
    const int g = nblocks(n);
    hipLaunchKernelGGL(k_multidot, dim3(g), dim3(kBlock), 0, s, n, V, ld, nv, w, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_multi_reduce, dim3(nv), dim3(kBlock), 0, s, partial, g, out);
    return hipGetLastError();
}

hipError_t launch_multi_axpy(long n, const double *V, long ld, int nv, const double *c, double a,
                             double *w, hipStream_t s)
{
    NMG_LAUNCH(k_multi_axpy, nblocks(n), n, V, ld, nv, c, a, w);
}

hipError_t launch_average(int dim, int nxf, int nyf, int ncomp, const double *f, double *c,
                          hipStream_t s)
{
    const long Nc = (long)(nxf / 2) * (dim == 1 ? 1 : nyf / 2);
    NMG_LAUNCH(k_average, nblocks(Nc), dim, nxf, nyf, ncomp, f, c);
}

hipError_t launch_inject(int dim, int nxf, int nyf, int ncomp, const double *c, double *f,
                         hipStream_t s)
{
    NMG_LAUNCH(k_inject, nblocks((long)nxf * nyf), dim, nxf, nyf, ncomp, c, f);
}

// ---- batched launchers ----

#define NMG_BLAUNCH(kern, ...)                                                         \
    do {                                                                               \
        if (w.n <= 0) return hipSuccess;                                               \
        hipLaunchKernelGGL(kern, dim3(w.n), dim3(kBlock), 0, s, __VA_ARGS__);          \
        return hipGetLastError();                                                      \
    } while (0)

hipError_t launch_b_isolated(int dim, const BatchInst *bi, WorkRange w, const int *active,
                             hipStream_t s)
{
    if (dim == 1) NMG_BLAUNCH(kb_isolated<2>, bi, w, active);
    NMG_BLAUNCH(kb_isolated<3>, bi, w, active);
}

hipError_t launch_b_assemble(int dim, bool f32, const BatchInst *bi, WorkRange w,
                             const int *active, double *partial, hipStream_t s)
{
    if (f32) {
        if (dim == 1) NMG_BLAUNCH((kb_assemble<2, float>), bi, w, active, partial);
        NMG_BLAUNCH((kb_assemble<3, float>), bi, w, active, partial);
    }
    if (dim == 1) NMG_BLAUNCH((kb_assemble<2, double>), bi, w, active, partial);
    NMG_BLAUNCH((kb_assemble<3, double>), bi, w, active, partial);
}

hipError_t launch_b_residual(int dim, const BatchInst *bi, WorkRange w, const int *active,
                             double *partial, hipStream_t s)
{
    if (dim == 1) NMG_BLAUNCH(kb_residual<2>, bi, w, active, partial);
    NMG_BLAUNCH(kb_residual<3>, bi, w, active, partial);
}

hipError_t launch_b_count_iso(const BatchInst *bi, WorkRange w, const int *active,
                              double *partial, hipStream_t s)
{
    NMG_BLAUNCH(kb_count_iso, bi, w, active, partial);
}

hipError_t launch_b_reduce(const double *partial, const int *off, const int *cnt, int n,
                           const int *active, double *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(kb_reduce, dim3(n), dim3(kBlock), 0, s, partial, off, cnt, active, out);
    return hipGetLastError();
}

hipError_t launch_b_blu_half(int dim, const BatchInst *bi, WorkRange w, const int *active,
                             int color, hipStream_t s)
{
    if (dim == 1) NMG_BLAUNCH(kb_blu_half<2>, bi, w, active, color);
    NMG_BLAUNCH(kb_blu_half<3>, bi, w, active, color);
}

hipError_t launch_b_update(int dim, bool f32, const BatchInst *bi, WorkRange w,
                           const int *active, hipStream_t s)
{
    if (f32) {
        if (dim == 1) NMG_BLAUNCH((kb_update<2, float>), bi, w, active);
        NMG_BLAUNCH((kb_update<3, float>), bi, w, active);
    }
    if (dim == 1) NMG_BLAUNCH((kb_update<2, double>), bi, w, active);
    NMG_BLAUNCH((kb_update<3, double>), bi, w, active);
}

hipError_t launch_b_threshold(int dim, const BatchInst *bi, WorkRange w, const int *active,
                              hipStream_t s)
{
    if (dim == 1) NMG_BLAUNCH(kb_threshold<2>, bi, w, active);
    NMG_BLAUNCH(kb_threshold<3>, bi, w, active);
}

hipError_t launch_b_copy_state(int dim, const BatchInst *bi, WorkRange w, const int *active,
                               int dir, hipStream_t s)
{
    if (dim == 1) NMG_BLAUNCH(kb_copy_state<2>, bi, w, active, dir);
    NMG_BLAUNCH(kb_copy_state<3>, bi, w, active, dir);
}

// persist > 0: the persistent form with that many blocks (at most one per
// work item).
template <class T, int NC, int TB>
static hipError_t bsgs_mode(int mode, const BatchLevel *lv, WorkRange w, const int *active,
                            int color, int persist, hipStream_t s)
{
    if (w.n <= 0) return hipSuccess;
    if (persist > 0) {
        const dim3 g(std::min(w.n, persist));
        switch (mode) {
        case MODE_NORMAL:
            hipLaunchKernelGGL((kb_sgs_half_loop<T, NC, MODE_NORMAL, TB>), g, dim3(TB), 0, s, lv, w, active, color);
            break;
        case MODE_ZERO:
            hipLaunchKernelGGL((kb_sgs_half_loop<T, NC, MODE_ZERO, TB>), g, dim3(TB), 0, s, lv, w, active, color);
            break;
        case MODE_PROLONG:
            hipLaunchKernelGGL((kb_sgs_half_loop<T, NC, MODE_PROLONG, TB>), g, dim3(TB), 0, s, lv, w, active, color);
            break;
        default:
            hipLaunchKernelGGL((kb_sgs_half_loop<T, NC, MODE_PROLONG_ZERO, TB>), g, dim3(TB), 0, s, lv, w, active, color);
            break;
        }
        return hipGetLastError();
    }
    switch (mode) {
    case MODE_NORMAL:
        hipLaunchKernelGGL((kb_sgs_half<T, NC, MODE_NORMAL, TB>), dim3(w.n), dim3(TB), 0, s, lv, w, active, color);
        break;
    case MODE_ZERO:
        hipLaunchKernelGGL((kb_sgs_half<T, NC, MODE_ZERO, TB>), dim3(w.n), dim3(TB), 0, s, lv, w, active, color);
        break;
    case MODE_PROLONG:
        hipLaunchKernelGGL((kb_sgs_half<T, NC, MODE_PROLONG, TB>), dim3(w.n), dim3(TB), 0, s, lv, w, active, color);
        break;
    default:
        hipLaunchKernelGGL((kb_sgs_half<T, NC, MODE_PROLONG_ZERO, TB>), dim3(w.n), dim3(TB), 0, s, lv, w, active, color);
        break;
    }
    return hipGetLastError();
}

template <class T, int NC>
static hipError_t bsgs_tile(int mode, int tile, const BatchLevel *lv, WorkRange w,
                            const int *active, int color, int persist, hipStream_t s)
{
    switch (tile) {
    case 64: return bsgs_mode<T, NC, 64>(mode, lv, w, active, color, persist, s);
    case 128: return bsgs_mode<T, NC, 128>(mode, lv, w, active, color, persist, s);
    case 256: return bsgs_mode<T, NC, 256>(mode, lv, w, active, color, persist, s);
    case 512: return bsgs_mode<T, NC, 512>(mode, lv, w, active, color, persist, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_b_sgs_half(int dim, bool f32, int mode, int tile, const BatchLevel *lv,
                             WorkRange w, const int *active, int color, int persist,
                             hipStream_t s)
{
    if (f32) {
        if (dim == 1) return bsgs_tile<float, 2>(mode, tile, lv, w, active, color, persist, s);
        return bsgs_tile<float, 3>(mode, tile, lv, w, active, color, persist, s);
    }
    if (dim == 1) return bsgs_tile<double, 2>(mode, tile, lv, w, active, color, persist, s);
    return bsgs_tile<double, 3>(mode, tile, lv, w, active, color, persist, s);
}

template <class T>
static hipError_t b_pair_dispatch(int mode, const BatchLevel *lv, WorkRange w, const int *active,
                                  int color, int flip, hipStream_t s)
{
#define NMG_BPAIR(M)                                                                          \
    do {                                                                                      \
        hipLaunchKernelGGL((kb_sgs_pair<T, M>), dim3(w.n), dim3(kPairThreads), 0, s, lv, w,   \
                           active, color, flip);                                              \
        return hipGetLastError();                                                             \
    } while (0)
    switch (mode) {
    case MODE_NORMAL: NMG_BPAIR(MODE_NORMAL);
    case MODE_ZERO: NMG_BPAIR(MODE_ZERO);
    case MODE_PROLONG: NMG_BPAIR(MODE_PROLONG);
    default: NMG_BPAIR(MODE_PROLONG_ZERO);
    }
#undef NMG_BPAIR
}

hipError_t launch_b_sgs_pair(bool f32, int mode, const BatchLevel *lv, WorkRange w,
                             const int *active, int color, int flip, hipStream_t s)
{
    if (w.n == 0) return hipSuccess;
    if (f32) return b_pair_dispatch<float>(mode, lv, w, active, color, flip, s);
    return b_pair_dispatch<double>(mode, lv, w, active, color, flip, s);
}

hipError_t launch_b_restrict(int dim, bool f32, const BatchLevel *lv, WorkRange w,
                             const int *active, hipStream_t s)
{
    if (f32) {
        if (dim == 1) NMG_BLAUNCH((kb_restrict<float, 2>), lv, w, active);
        NMG_BLAUNCH((kb_restrict<float, 3>), lv, w, active);
    }
    if (dim == 1) NMG_BLAUNCH((kb_restrict<double, 2>), lv, w, active);
    NMG_BLAUNCH((kb_restrict<double, 3>), lv, w, active);
}

hipError_t launch_b_restrict_res(int dim, bool f32, const BatchLevel *lv, WorkRange w,
                                 const int *active, int rcol, hipStream_t s)
{
    if (f32) {
        if (dim == 1) NMG_BLAUNCH((kb_restrict_res<float, 2>), lv, w, active, rcol);
        NMG_BLAUNCH((kb_restrict_res<float, 3>), lv, w, active, rcol);
    }
    if (dim == 1) NMG_BLAUNCH((kb_restrict_res<double, 2>), lv, w, active, rcol);
    NMG_BLAUNCH((kb_restrict_res<double, 3>), lv, w, active, rcol);
}

template <class T, int NC>
static hipError_t bsgs_res_tile(int tile, const BatchLevel *lv, WorkRange w, const int *active,
                                int color, hipStream_t s)
{
    if (w.n <= 0) return hipSuccess;
#define NMG_BRES(TB)                                                                          \
    hipLaunchKernelGGL((kb_sgs_half_res<T, NC, TB>), dim3(w.n), dim3(TB), 0, s, lv, w, active, \
                       color);                                                                \
    return hipGetLastError()
    switch (tile) {
    case 64: NMG_BRES(64);
    case 128: NMG_BRES(128);
    case 256: NMG_BRES(256);
    case 512: NMG_BRES(512);
    default: return hipErrorInvalidValue;
    }
#undef NMG_BRES
}

hipError_t launch_b_sgs_half_res(int dim, bool f32, int tile, const BatchLevel *lv, WorkRange w,
                                 const int *active, int color, hipStream_t s)
{
    if (f32) {
        if (dim == 1) return bsgs_res_tile<float, 2>(tile, lv, w, active, color, s);
        return bsgs_res_tile<float, 3>(tile, lv, w, active, color, s);
    }
    if (dim == 1) return bsgs_res_tile<double, 2>(tile, lv, w, active, color, s);
    return bsgs_res_tile<double, 3>(tile, lv, w, active, color, s);
}

hipError_t launch_b_fix_color(int dim, bool f32, int op, const BatchLevel *lv, WorkRange w,
                              const int *active, int color, hipStream_t s)
{
    if (f32) {
        if (dim == 1) NMG_BLAUNCH((kb_fix_color<float, 2>), lv, w, active, op, color);
        NMG_BLAUNCH((kb_fix_color<float, 3>), lv, w, active, op, color);
    }
    if (dim == 1) NMG_BLAUNCH((kb_fix_color<double, 2>), lv, w, active, op, color);
    NMG_BLAUNCH((kb_fix_color<double, 3>), lv, w, active, op, color);
}

hipError_t launch_b_galerkin(int dim, bool f32, const BatchLevel *lv, WorkRange w,
                             const int *active, hipStream_t s)
{
    if (f32) {
        if (dim == 1) NMG_BLAUNCH((kb_galerkin<float, 2>), lv, w, active);
        NMG_BLAUNCH((kb_galerkin<float, 3>), lv, w, active);
    }
    if (dim == 1) NMG_BLAUNCH((kb_galerkin<double, 2>), lv, w, active);
    NMG_BLAUNCH((kb_galerkin<double, 3>), lv, w, active);
}

hipError_t launch_b_coarse_cycle(int dim, bool f32, const CoarseOp *ops, int nops,
                                 const LevelDev *lv, int ninst, const int *active, int l_lds,
                                 int nl, hipStream_t s)
{
    if (ninst <= 0) return hipSuccess;
#define NMG_BCOARSE(T, NC)                                                                    \
    do {                                                                                      \
        hipLaunchKernelGGL((k_coarse_cycle<T, NC>), dim3(ninst), dim3(kCoarseBlock), 0, s,    \
                           ops, nops, lv, active, l_lds, nl);                                 \
        return hipGetLastError();                                                             \
    } while (0)
    if (f32) {
        if (dim == 1) NMG_BCOARSE(float, 2);
        NMG_BCOARSE(float, 3);
    }
    if (dim == 1) NMG_BCOARSE(double, 2);
    NMG_BCOARSE(double, 3);
#undef NMG_BCOARSE
}

hipError_t launch_vec_to_split(int nc, bool f32, const LevelGeom &G, const double *v, void *split,
                               hipStream_t s)
{
    int g = nblocks((long)G.nx * G.ny);
    if (f32) NMG_LAUNCH(k_to_split<float>, g, nc, G, v, (float *)split);
    NMG_LAUNCH(k_to_split<double>, g, nc, G, v, (double *)split);
}

hipError_t launch_vec_from_split(int nc, bool f32, const LevelGeom &G, const void *split,
                                 double *v, hipStream_t s)
{
    int g = nblocks((long)G.nx * G.ny);
    if (f32) NMG_LAUNCH(k_from_split<float>, g, nc, G, (const float *)split, v);
    NMG_LAUNCH(k_from_split<double>, g, nc, G, (const double *)split, v);
}

hipError_t launch_mat_to_split(int ne, bool f32, const LevelGeom &G, const double *A, void *split,
                               hipStream_t s)
{
    int g = nblocks((long)G.nx * G.ny);
    if (f32) NMG_LAUNCH(k_mat_to_tiled<float>, g, ne, G, A, (float *)split);
    NMG_LAUNCH(k_mat_to_tiled<double>, g, ne, G, A, (double *)split);
}

hipError_t launch_mat_from_split(int ne, bool f32, const LevelGeom &G, const void *split,
                                 double *A, hipStream_t s)
{
    int g = nblocks((long)G.nx * G.ny);
    if (f32) NMG_LAUNCH(k_mat_from_tiled<float>, g, ne, G, (const float *)split, A);
    NMG_LAUNCH(k_mat_from_tiled<double>, g, ne, G, (const double *)split, A);
}

}  // namespace nmg
