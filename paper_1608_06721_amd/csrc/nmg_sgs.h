// Block solve and red-black block Gauss-Seidel half sweep (Sec. 2.3: the
// smoother of the multigrid cycle) on the colour-split layout, shared by the
// per-level launches and the single-workgroup coarse-cycle kernel.
//
// Compiled with -ffp-contract=off: the order of every floating-point
// expression is fixed, so results are bit-for-bit deterministic.
#pragma once

#include "nmg_internal.h"

#include <hip/hip_runtime.h>

namespace nmg {
namespace {

// Faces of a cell: west, east, south, north (1D uses W and E).
enum { FW = 0, FE = 1, FS = 2, FN = 3 };

// XCD-aware block order.  Workgroups are dispatched round-robin over the
// chip's 8 XCDs, each with its own L2.  Renumbering so that XCD b % 8 takes
// chunks of kXcdChunk consecutive tiles (16 rows of a 1024-wide level) keeps
// neighbouring rows of a stencil in one L2, so values shared between rows
// are fetched from HBM once, while the 8 XCDs still stream nearby addresses.
// Blocks past the last full group of 8 chunks keep their number; a bijection
// on [0, n) for any n.
constexpr int kXcds = 8;
constexpr int kXcdChunk = 32;
__device__ __forceinline__ int xcd_block(int b, int n)
{
    constexpr int G = kXcds * kXcdChunk;
    if (b >= n / G * G) return b;
    const int x = b % kXcds, k = b / kXcds;
    return (k / kXcdChunk) * G + x * kXcdChunk + k % kXcdChunk;
}

// Load of matrix data that one launch reads exactly once, on a level large
// enough that the host streams it (stream_level).  In FP64 the off-diagonal
// blocks are then fetched with the non-temporal hint (measured: the
// 1024x1024 half sweep runs 13% faster; in FP32, and for the diagonal block
// and b, the hint is slower or neutral).
template <class T, bool STREAM>
__device__ __forceinline__ T ld_once(const T *p)
{
    if constexpr (STREAM && sizeof(T) == 8) return __builtin_nontemporal_load(p);
    else return *p;
}

// Solve the NC x NC block system D x = r in precision T: adjugate (cofactors
// along row 0) times the reciprocal determinant; x = 0 when that reciprocal
// is not finite.
template <class T, int NC>
__device__ __forceinline__ void solve_block(const T *D, const T *r, T *x)
{
    if (NC == 2) {
        T det = D[0] * D[3] - D[1] * D[2];
        T idet = T(1) / det;
        if (!__builtin_isfinite(idet)) { x[0] = T(0); x[1] = T(0); return; }
        x[0] = (D[3] * r[0] - D[1] * r[1]) * idet;
        x[1] = (D[0] * r[1] - D[2] * r[0]) * idet;
        return;
    }
    T d00 = D[0], d01 = D[1], d02 = D[2];
    T d10 = D[3], d11 = D[4], d12 = D[5];
    T d20 = D[6], d21 = D[7], d22 = D[8];
    T C00 = d11 * d22 - d12 * d21, C01 = d12 * d20 - d10 * d22, C02 = d10 * d21 - d11 * d20;
    T C10 = d02 * d21 - d01 * d22, C11 = d00 * d22 - d02 * d20, C12 = d01 * d20 - d00 * d21;
    T C20 = d01 * d12 - d02 * d11, C21 = d02 * d10 - d00 * d12, C22 = d00 * d11 - d01 * d10;
    T det = d00 * C00 + d01 * C01 + d02 * C02;
    T idet = T(1) / det;
    if (!__builtin_isfinite(idet)) { x[0] = T(0); x[1] = T(0); x[2] = T(0); return; }
    x[0] = (C00 * r[0] + C10 * r[1] + C20 * r[2]) * idet;
    x[1] = (C01 * r[0] + C11 * r[1] + C21 * r[2]) * idet;
    x[2] = (C02 * r[0] + C12 * r[1] + C22 * r[2]) * idet;
}

// Precomputed form of solve_block for blocks that many sweeps reuse: the
// cofactors in the order the solution products read them and the reciprocal
// determinant (NaN marks a block whose reciprocal is not finite).  Applying
// it with solve_inv performs solve_block's final products and sums in the
// same order, so the result is bit-for-bit the same.
template <class T, int NC>
__device__ __forceinline__ void block_inverse(const T *D, T *inv)
{
    const T nan = T(__builtin_nan(""));
    if (NC == 2) {
        T det = D[0] * D[3] - D[1] * D[2];
        T idet = T(1) / det;
        inv[0] = D[3]; inv[1] = D[1]; inv[2] = D[0]; inv[3] = D[2];
        inv[4] = __builtin_isfinite(idet) ? idet : nan;
        return;
    }
    T d00 = D[0], d01 = D[1], d02 = D[2];
    T d10 = D[3], d11 = D[4], d12 = D[5];
    T d20 = D[6], d21 = D[7], d22 = D[8];
    T C00 = d11 * d22 - d12 * d21, C01 = d12 * d20 - d10 * d22, C02 = d10 * d21 - d11 * d20;
    T C10 = d02 * d21 - d01 * d22, C11 = d00 * d22 - d02 * d20, C12 = d01 * d20 - d00 * d21;
    T C20 = d01 * d12 - d02 * d11, C21 = d02 * d10 - d00 * d12, C22 = d00 * d11 - d01 * d10;
    T det = d00 * C00 + d01 * C01 + d02 * C02;
    T idet = T(1) / det;
    inv[0] = C00; inv[1] = C10; inv[2] = C20;
    inv[3] = C01; inv[4] = C11; inv[5] = C21;
    inv[6] = C02; inv[7] = C12; inv[8] = C22;
    inv[9] = __builtin_isfinite(idet) ? idet : nan;
}

template <class T, int NC>
__device__ __forceinline__ void solve_inv(const T *inv, const T *r, T *x)
{
    const T idet = inv[NC * NC];
    const bool sing = idet != idet;
    if (NC == 2) {
        x[0] = (inv[0] * r[0] - inv[1] * r[1]) * idet;
        x[1] = (inv[2] * r[1] - inv[3] * r[0]) * idet;
    } else {
#pragma unroll
        for (int k = 0; k < NC; ++k)
            x[k] = (inv[3 * k] * r[0] + inv[3 * k + 1] * r[1] + inv[3 * k + 2] * r[2]) * idet;
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) x[k] = sing ? T(0) : x[k];
}

// Value of the other-colour neighbour at fine cell (ni, nj) under `mode`.
template <class T, int NC, int MODE>
__device__ __forceinline__ void read_other(const LevelGeom &G, const T *xo, int ni, int nj,
                                           const LevelGeom &Gc, const T *xc, T *v)
{
    if (MODE == MODE_ZERO) {
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = T(0);
        return;
    }
    T base[NC];
    if (MODE == MODE_NORMAL || MODE == MODE_PROLONG) {
        const T *p = xo + (long)nj * G.W + (ni >> 1);
#pragma unroll
        for (int c = 0; c < NC; ++c) base[c] = p[c * G.plane];
    } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) base[c] = T(0);
    }
    if (MODE == MODE_NORMAL) {
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = base[c];
        return;
    }
    int I = ni >> 1, J = nj >> 1;
    int cc = (I + J) & 1;
    const T *p = xc + (long)cc * NC * Gc.plane + (long)J * Gc.W + (I >> 1);
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = base[c] + p[c * Gc.plane];
}

// The arithmetic of one block Gauss-Seidel cell update: acc = sum over the
// neighbours (W, E, S, N order) and components of A_f x_f, then
// x_i = D_i^-1 (b_i - acc) by solve_block (a holds D) or solve_inv (inv).
// ZERO: every neighbour value is zero, so acc = 0.  A face without a
// neighbour has a zero block and a zero value here, so its terms are +0 and
// leave acc unchanged (acc starts at +0 and can never become -0): it is
// summed like the others, without a branch.  Each row's sum runs in face,
// then component order; the rows are interleaved.
template <class T, int NC, bool ZERO, bool INV>
__device__ __forceinline__ void gs_update(const T *a, const T *inv, const T *bv,
                                          const T (*v)[NC], const bool *ok, T *xi)
{
    constexpr int NF = (NC == 2) ? 2 : 4;
    (void)ok;
    T acc[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r) acc[r] = T(0);
    if (!ZERO) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            T p[NC][NC];
#pragma unroll
            for (int r = 0; r < NC; ++r)
#pragma unroll
                for (int c = 0; c < NC; ++c) p[r][c] = a[((f + 1) * NC + r) * NC + c] * v[f][c];
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int r = 0; r < NC; ++r) acc[r] = acc[r] + p[r][c];
        }
    }
    T rhs[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r) rhs[r] = bv[r] - acc[r];
    if (INV)
        solve_inv<T, NC>(inv, rhs, xi);
    else
        solve_block<T, NC>(a, rhs, xi);
}

// Block Gauss-Seidel half sweep of one colour: x_i = D_i^-1 (b_i - sum_j
// A_ij x_j), the sum over existing neighbours in W, E, S, N order and then
// components.  One thread per cell of the colour, coalesced along x.  All
// loads of a cell (its block row, b_i and the neighbours' x) are issued
// before any arithmetic, so each wave keeps ~50 independent loads in flight.
// INV: the diagonal block is applied through its precomputed inverse data
// Ai (tiled like A, inv_entries(NC) entries per slot) instead of solve_block.
// STREAM: off-diagonal blocks loaded through ld_once.
// RES (normal mode, INV false): also write the cell's linear residual after
// its update, b_i - (D_i x_i + sum over existing faces A_ij x_j) in the
// order of the restriction's residual, to rout (NC planes of the colour's
// slots): the other colour is unchanged until the next half sweep, so it is
// bit for bit the residual the restriction would compute.
template <class T, int NC, int MODE, bool INV = false, bool STREAM = false, bool RES = false>
__device__ __forceinline__ void sgs_cell(const LevelGeom &G, const T *__restrict__ A,
                                         const T *__restrict__ Ai,
                                         const T *__restrict__ b, T *__restrict__ x,
                                         int color, const LevelGeom &Gc,
                                         const T *__restrict__ xc, long t,
                                         T *__restrict__ rout = nullptr)
{
    static_assert(!RES || (MODE == MODE_NORMAL && !INV), "residual output needs D and x_j");
    constexpr int NF = (NC == 2) ? 2 : 4;
    constexpr int NN = NC * NC;
    constexpr int NE = (NF + 1) * NN;
    constexpr int NI = inv_entries(NC);
    const int j = (int)(t / G.W), k = (int)(t % G.W);
    const int i = 2 * k + ((j + color) & 1);
    if (i >= G.nx) return;
    const int oc = color ^ 1;
    const T *Am = A + mat_off(G, NE, color, t);
    const T *bm = b + (long)color * NC * G.plane + t;
    const T *xo = x + (long)oc * NC * G.plane;

    bool ok[NF];
    int ni[NF], nj[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        ni[f] = i;
        nj[f] = j;
        if (f == FW) { ni[f] = i - 1; ok[f] = i > 0; }
        else if (f == FE) { ni[f] = i + 1; ok[f] = i + 1 < G.nx; }
        else if (f == FS) { nj[f] = j - 1; ok[f] = j > 0; }
        else { nj[f] = j + 1; ok[f] = j + 1 < G.ny; }
    }
    T a[NE], bv[NC], v[NF][NC], inv[NI];
    if (INV) {
        const T *Im = Ai + mat_off(G, NI, color, t);
#pragma unroll
        for (int e = 0; e < NI; ++e) inv[e] = Im[e * kTile];
    } else {
#pragma unroll
        for (int e = 0; e < NN; ++e) a[e] = Am[e * kTile];
    }
#pragma unroll
    for (int r = 0; r < NC; ++r) bv[r] = bm[r * G.plane];
    if (MODE != MODE_ZERO) {
#pragma unroll
        for (int e = NN; e < NE; ++e) a[e] = ld_once<T, STREAM>(&Am[e * kTile]);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            if (ok[f]) {
                read_other<T, NC, MODE>(G, xo, ni[f], nj[f], Gc, xc, v[f]);
            } else {
#pragma unroll
                for (int c = 0; c < NC; ++c) v[f][c] = T(0);
            }
        }
    }
    T xi[NC];
    gs_update<T, NC, MODE == MODE_ZERO, INV>(a, inv, bv, v, ok, xi);
    T *xm = x + (long)color * NC * G.plane + t;
#pragma unroll
    for (int r = 0; r < NC; ++r) xm[r * G.plane] = xi[r];
    if constexpr (RES) {
        T acc[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            acc[q] = T(0);
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[q] = acc[q] + a[q * NC + c] * xi[c];
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            if (!ok[f]) continue;
#pragma unroll
            for (int q = 0; q < NC; ++q)
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    acc[q] = acc[q] + a[((f + 1) * NC + q) * NC + c] * v[f][c];
        }
#pragma unroll
        for (int q = 0; q < NC; ++q) rout[q * G.plane + t] = bv[q] - acc[q];
    }
}

template <class T, int NC, int MODE, bool STREAM>
__global__ void __launch_bounds__(kBlock) k_sgs_half(LevelGeom G, const T *__restrict__ A,
                                                     const T *__restrict__ b,
                                                     T *__restrict__ x, int color,
                                                     LevelGeom Gc, const T *__restrict__ xc)
{
    long t = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (t >= G.plane) return;
    sgs_cell<T, NC, MODE, false, STREAM>(G, A, nullptr, b, x, color, Gc, xc, t);
}

// A normal-mode half sweep that also writes its cells' residuals to rout.
template <class T, int NC, bool STREAM>
__global__ void __launch_bounds__(kBlock) k_sgs_half_res(LevelGeom G, const T *__restrict__ A,
                                                         const T *__restrict__ b,
                                                         T *__restrict__ x, int color,
                                                         T *__restrict__ rout)
{
    long t = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (t >= G.plane) return;
    sgs_cell<T, NC, MODE_NORMAL, false, STREAM, true>(G, A, nullptr, b, x, color, G, nullptr, t,
                                                      rout);
}

}  // namespace
}  // namespace nmg
