"""Plain NumPy TT-cross and maxvol (Sec. IV.A and IV.B).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The method builds a tensor train (matrix product state, Sec. IV.A) of the
integrand tensor A[i_1..i_d] from entries only. Sec. IV.B describes it as an
iterated matrix cross: M ~ M(:,J) M(I,J)^{-1} M(I,:) with the rows I chosen for
large |det M(I,J)| by the maxvol heuristic, solving one matrix cross problem per
core while the other links are held fixed, sweeping back and forth.

Steps implemented here (one-site cross with orthogonalisation, the form used in
the TT-cross literature the paper cites):

  left-to-right, core k = 0..d-2:
    F[(a,i), b] = A[I_k[a], i, J_{k+1}[b]]        rows: left set x node, cols: right set
    append p random right multi-indices as extra columns (rank enrichment)
    R = triangular factor of a QR of F
    column-pivoted QR of R: R P = Q2 R2; keep r = #{|R2_jj| > eps_r |R2_00|} (<= max_rank)
    Y = F P[:, :r] R2[:r,:r]^{-1}                   orthonormal basis of the kept columns
    rows = maxvol(Y);  G_k = Y Y[rows]^{-1}          interpolating core, G_k[rows] = I
    I_{k+1} = {(I_k[a], i) for (a, i) in rows}
  last core G_{d-1}[a, i] = A[I_{d-1}[a], i]
  right-to-left: the mirror image, producing the right sets J_k.
  After every half sweep the quadrature sum P = 1^T M_0 ... M_{d-1} 1 with
  M_k = sum_i G_k[:, i, :] is formed; stop when |dP| <= tol |P|.

maxvol follows Goreinov-Tyrtyshnikov: start from the pivots of Gaussian
elimination with partial pivoting, then repeatedly swap in the entry of largest
modulus of B = Y Y[rows]^{-1} while it exceeds 1 + delta (rank-one update of B).

Parity: maxvol is pinned against exhaustive search on small matrices; the TT
sum is pinned against the dense Fourier sum (tests/test_oracle_ttcross.py).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def maxvol(A, delta=1e-2, max_swaps=None):
    """Rows of a dominant r x r submatrix of the m x r matrix A, and B = A A[rows]^{-1}."""
    A = np.asarray(A)
    m, r = A.shape
    # initial rows: Gaussian elimination with partial pivoting
    W = A.astype(complex).copy()
    rows = []
    free = np.ones(m, bool)
    for j in range(r):
        col = np.abs(W[:, j])
        col[~free] = -1.0
        i = int(np.argmax(col))
        rows.append(i)
        free[i] = False
        if W[i, j] != 0:
            W -= np.outer(W[:, j] / W[i, j], W[i, :]) * (np.arange(r) >= j)[None, :]
    rows = np.array(rows)
    B = np.linalg.solve(A[rows].T, A.T).T
    if max_swaps is None:
        max_swaps = 4 * r + 16
    for _ in range(max_swaps):
        absB = np.abs(B)
        flat = int(np.argmax(absB))
        i, j = divmod(flat, r)
        if absB[i, j] <= 1.0 + delta:
            break
        bij = B[i, j]
        ej = np.zeros(r, B.dtype)
        ej[j] = 1.0
        B = B - np.outer(B[:, j], (B[i, :] - ej) / bij)
        rows[j] = i
    return rows, B


def _basis(F, eps_r, max_rank):
    R = np.linalg.qr(F, mode="r")
    _, R2, perm = sla.qr(R, pivoting=True)
    dg = np.abs(np.diag(R2))
    if dg[0] == 0:
        r = 1
    else:
        r = int(np.sum(dg > eps_r * dg[0]))
    r = max(1, min(r, max_rank))
    Y = sla.solve_triangular(R2[:r, :r].T, F[:, perm[:r]].T, lower=True).T
    return Y, r


def tt_contract(cores, weights=None):
    """sum over all indices of the TT times prod_k weights[k][i_k]."""
    v = np.ones((1,), complex)
    for k, G in enumerate(cores):
        w = np.ones(G.shape[1]) if weights is None else weights[k]
        M = np.einsum("aib,i->ab", G, w)
        v = v @ M
    return v[0]


def tt_value(cores, idx):
    idx = np.atleast_2d(idx)
    out = np.empty(idx.shape[0], complex)
    for p in range(idx.shape[0]):
        v = np.ones((1,), complex)
        for k, G in enumerate(cores):
            v = v @ G[:, idx[p, k], :]
        out[p] = v[0]
    return out


def tt_cross(fun, d, N, max_rank, tol, max_sweeps=6, seed=0, n_enrich=4, eps_rank=None,
             init_rank=None):
    """fun(idx[n, d] int) -> complex values. Returns (cores, info)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if eps_rank is None:
        eps_rank = tol / np.sqrt(max(d - 1, 1)) * 0.1
    r0 = max_rank if init_rank is None else init_rank
    # rank caps per bond from the tensor shape
    cap = [1] + [int(min(max_rank, N ** min(k, d - k), 10 ** 9)) for k in range(1, d)] + [1]
    # right sets J[k] for k = 1..d-1: multi-indices over coords k..d-1, drawn near the grid centre
    J = [None] * (d + 1)
    J[d] = np.zeros((1, 0), int)
    for k in range(d - 1, 0, -1):
        rk = min(r0, cap[k])
        J[k] = np.concatenate([rng.integers(N // 4, 3 * N // 4, size=(rk, 1)),
                               J[k + 1][rng.integers(0, J[k + 1].shape[0], size=rk)]], axis=1)
    I = [None] * (d + 1)
    I[0] = np.zeros((1, 0), int)
    cores = [None] * d
    history = []
    n_evals = 0
    rank_capped = False
    converged = False
    P_prev = None
    sweeps = 0

    def fiber(Ik, k, Jk1):
        ra, rb = Ik.shape[0], Jk1.shape[0]
        a = np.repeat(np.arange(ra), N * rb)
        i = np.tile(np.repeat(np.arange(N), rb), ra)
        b = np.tile(np.arange(rb), ra * N)
        idx = np.concatenate([Ik[a], i[:, None], Jk1[b]], axis=1)
        return fun(idx).reshape(ra, N, rb)

    for sweep in range(max_sweeps):
        sweeps = sweep + 1
        # ---------------- left to right
        for k in range(d - 1):
            Jx = J[k + 1]
            extra = np.concatenate([rng.integers(0, N, size=(n_enrich, d - k - 1))], axis=1)
            Jx = np.concatenate([Jx, extra], axis=0)
            Fk = fiber(I[k], k, Jx)
            n_evals += Fk.size
            ra = I[k].shape[0]
            F = Fk.reshape(ra * N, Jx.shape[0])
            Y, r = _basis(F, eps_rank, min(max_rank, cap[k + 1], ra * N))
            if r == min(max_rank, cap[k + 1]) and r < ra * N:
                rank_capped = True
            rows, B = maxvol(Y)
            cores[k] = B.reshape(ra, N, r)
            I[k + 1] = np.concatenate([I[k][rows // N], (rows % N)[:, None]], axis=1)
        Fd = fiber(I[d - 1], d - 1, J[d])
        n_evals += Fd.size
        cores[d - 1] = Fd
        P = tt_contract(cores)
        history.append(P)
        if P_prev is not None and abs(P - P_prev) <= tol * abs(P):
            converged = True
            break
        P_prev = P
        # ---------------- right to left
        for k in range(d - 1, 0, -1):
            Ix = I[k]
            extra = rng.integers(0, N, size=(n_enrich, k))
            Ix = np.concatenate([Ix, extra], axis=0)
            Fk = fiber(Ix, k, J[k + 1])
            n_evals += Fk.size
            rb = J[k + 1].shape[0]
            F = Fk.reshape(Ix.shape[0], N * rb).T      # rows (i, b), cols a
            Y, r = _basis(F, eps_rank, min(max_rank, cap[k], N * rb))
            if r == min(max_rank, cap[k]) and r < N * rb:
                rank_capped = True
            rows, B = maxvol(Y)
            cores[k] = B.T.reshape(r, N, rb)
            J[k] = np.concatenate([(rows // rb)[:, None], J[k + 1][rows % rb]], axis=1)
        F0 = fiber(I[0], 0, J[1])
        n_evals += F0.size
        cores[0] = F0
        P = tt_contract(cores)
        history.append(P)
        if abs(P - P_prev) <= tol * abs(P):
            converged = True
            break
        P_prev = P
    ranks = [1] + [c.shape[2] for c in cores[:-1]] + [1]
    return cores, dict(history=history, n_evals=n_evals, ranks=ranks, sweeps=sweeps,
                       converged=converged, rank_capped=rank_capped)
