"""Direct solvers used to pin the oracle (test infrastructure only).

* ``assemble_fine`` builds the finest-level discrete operator of the paper
  (Sec. 2 7-point Laplacian; Sec. 3 ghost value with the boundary on the face
  between an active and an inactive cell) as a sparse matrix, with the
  Dirichlet contribution moved to the right-hand side, and
  ``direct_solve`` solves it with a library factorisation.
* ``dst_solve_box`` solves the all-active box (one inactive frame layer,
  zero Dirichlet values) exactly with a type-II discrete sine transform: the
  modes sin(k pi (i + 1/2) / m) are eigenvectors of that operator.

Both are independent of ``mg_oracle.c`` (different language, no shared code).
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def assemble_fine(mask, h, dirichlet=None):
    """Return (A, b, ids): A x = b on active cells, ids maps flat index -> row.

    Row of active cell i:  (1/h^2) [ sum_{j active} (x_j - x_i)
                                   + sum_{j inactive} (ghost_ij - x_i) ] = rho_i
    with ghost_ij = 2 g_ij - x_i (linear extrapolation through x_i and the
    face value g_ij = (B_i + B_j)/2 placed half a cell away).
    The returned b excludes rho; the caller adds rho (b_total = rho - b).
    """
    mask = np.asarray(mask)
    nz, ny, nx = mask.shape
    act = (mask == 1).ravel()
    ids = -np.ones(act.size, dtype=np.int64)
    ids[act] = np.arange(int(act.sum()))
    B = None if dirichlet is None else np.asarray(dirichlet, dtype=np.float64).ravel()
    rows, cols, vals = [], [], []
    bnd = np.zeros(int(act.sum()))
    strides = {(-1, 0, 0): -1, (1, 0, 0): 1, (0, -1, 0): -nx, (0, 1, 0): nx, (0, 0, -1): -nx * ny, (0, 0, 1): nx * ny}
    ih2 = 1.0 / (h * h)
    for p in np.flatnonzero(act):
        k, rem = divmod(p, nx * ny)
        j, i = divmod(rem, nx)
        r = ids[p]
        diag = 0.0
        for (dx, dy, dz), s in strides.items():
            ii, jj, kk = i + dx, j + dy, k + dz
            q = p + s
            inb = 0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz
            if inb and act[q]:
                rows.append(r); cols.append(ids[q]); vals.append(ih2)
                diag -= ih2
            else:
                # ghost - x_i = 2 g - 2 x_i
                diag -= 2.0 * ih2
                if B is not None and inb:
                    bnd[r] += 2.0 * ih2 * 0.5 * (B[p] + B[q])
        rows.append(r); cols.append(r); vals.append(diag)
    n = int(act.sum())
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    return A, bnd, ids


def direct_solve(mask, h, rho, dirichlet=None, dense=False):
    """Exact discrete solution on active cells (inactive cells = 0)."""
    A, bnd, ids = assemble_fine(mask, h, dirichlet)
    act = ids >= 0
    b = np.asarray(rho, dtype=np.float64).ravel()[act] - bnd
    if dense:
        x = np.linalg.solve(A.toarray(), b)
    else:
        x = spla.spsolve(A.tocsc(), b)
    out = np.zeros(np.asarray(mask).size)
    out[act] = x
    return out.reshape(np.asarray(mask).shape)


def dst_solve_box(rho_inner, h):
    """Solve the all-active interior block (shape (mz, my, mx)) with zero
    Dirichlet values on its outer faces, exactly, by DST-II."""
    m = rho_inner.shape
    rk = scipy.fft.dstn(rho_inner, type=2, norm="ortho")
    lam = np.zeros(m)
    for axis, ma in enumerate(m):
        k = np.arange(1, ma + 1)
        s = -(4.0 / (h * h)) * np.sin(k * np.pi / (2 * ma)) ** 2
        sh = [1, 1, 1]
        sh[axis] = ma
        lam = lam + s.reshape(sh)
    return scipy.fft.idstn(rk / lam, type=2, norm="ortho")
