"""Test-side helpers: explicit sparse matrices built from stencil coefficients.

These build the textbook objects (the 7-point matrix, the restriction and
prolongation matrices) from plain index arithmetic so that the oracle can be
checked against SciPy's products and factorisations.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def stencil_matrix(pb, W, diag):
    """CSR matrix with A_ii = diag_i, A_ij = -W_f on the face between i, j."""
    nx, ny, nz = pb.nx, pb.ny, pb.nz
    N = pb.n
    idx = np.arange(N).reshape(nz, ny, nx)
    rows, cols, vals = [np.arange(N)], [np.arange(N)], [np.asarray(diag, dtype=np.float64)]
    Wx, Wy, Wz = (np.asarray(w).reshape(nz, ny, nx) for w in W)
    for w, a, b in ((Wx[:, :, :-1], idx[:, :, :-1], idx[:, :, 1:]),
                    (Wy[:, :-1, :], idx[:, :-1, :], idx[:, 1:, :]),
                    (Wz[:-1, :, :], idx[:-1, :, :], idx[1:, :, :])):
        w, a, b = w.ravel(), a.ravel(), b.ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [-w, -w]
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    A.sum_duplicates()
    return A


def prolongation_matrix(pb, P, slot_nodes, num_coarse):
    """Sparse P_hat (N x Nc) from slot weights, Dirichlet rows zeroed."""
    N = pb.n
    dm = pb.dirichlet_mask().astype(bool)
    rows, cols, vals = [], [], []
    for s in range(8):
        w = P[s].copy()
        w[dm] = 0.0
        keep = w != 0.0
        assert np.all(slot_nodes[s][keep] >= 0)
        rows.append(np.nonzero(keep)[0])
        cols.append(slot_nodes[s][keep])
        vals.append(w[keep])
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, num_coarse)).tocsr()


def fv_restriction_matrix(primal_block, num_coarse):
    N = primal_block.size
    return sp.coo_matrix((np.ones(N), (primal_block, np.arange(N))), shape=(num_coarse, N)).tocsr()


def direct_newton(pb, T, pn, p, tol=1e-12, maxit=50):
    """Newton with the paper's linearisation and a sparse direct solve."""
    import oracle
    import scipy.sparse.linalg as spla
    p = np.array(p, dtype=np.float64, copy=True)
    for it in range(maxit + 1):
        W, diag, r, e = oracle.linear_system(pb, T, p, pn)
        if e <= tol:
            return p, it
        A = stencil_matrix(pb, W, diag).tocsc()
        p = p + spla.splu(A).solve(r)
    raise RuntimeError("direct Newton did not converge")
