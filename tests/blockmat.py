"""Test-side bookkeeping: block-stencil arrays <-> dense matrices.

A is [nb][nc][nc][ny][nx] with blocks (D, W, E, S, N) (1D: D, W, E); the
unknown of cell (i, j) component c sits at dense index (j*nx + i)*nc + c.
"""
import numpy as np

OFFS = {0: (0, 0), 1: (-1, 0), 2: (1, 0), 3: (0, -1), 4: (0, 1)}


def dense(A):
    nb, nc, _, ny, nx = A.shape
    N = nx * ny
    M = np.zeros((nc * N, nc * N))
    for j in range(ny):
        for i in range(nx):
            c = j * nx + i
            for b in range(nb):
                di, dj = OFFS[b]
                ii, jj = i + di, j + dj
                if not (0 <= ii < nx and 0 <= jj < ny):
                    continue
                n = jj * nx + ii
                M[c * nc:(c + 1) * nc, n * nc:(n + 1) * nc] += A[b, :, :, j, i]
    return M


def vec(x):
    """[nc][ny][nx] -> dense vector (cell-major)."""
    nc = x.shape[0]
    return x.reshape(nc, -1).T.reshape(-1)


def unvec(v, nc, ny, nx):
    return v.reshape(ny * nx, nc).T.reshape(nc, ny, nx)


def prolongation(nc, ny, nx, dim):
    """Dense piecewise-constant prolongation from the coarse grid."""
    ncx, ncy = nx // 2, (ny // 2 if dim == 2 else 1)
    P = np.zeros((nc * nx * ny, nc * ncx * ncy))
    for j in range(ny):
        for i in range(nx):
            f = j * nx + i
            c = (j // 2 if dim == 2 else 0) * ncx + i // 2
            for k in range(nc):
                P[f * nc + k, c * nc + k] = 1.0
    return P


def block_split(M, nc, order):
    """Block diagonal, strictly lower and strictly upper parts of M with
    respect to the cell order `order` (a permutation of cell indices)."""
    n = M.shape[0] // nc
    pos = np.empty(n, dtype=int)
    pos[np.asarray(order)] = np.arange(n)
    D = np.zeros_like(M)
    L = np.zeros_like(M)
    U = np.zeros_like(M)
    for a in range(n):
        for c in range(n):
            blk = M[a * nc:(a + 1) * nc, c * nc:(c + 1) * nc]
            if not blk.any():
                continue
            tgt = D if a == c else (L if pos[c] < pos[a] else U)
            tgt[a * nc:(a + 1) * nc, c * nc:(c + 1) * nc] = blk
    return D, L, U
