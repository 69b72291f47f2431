"""Block BiCGStab on the even-odd system, s right-hand sides sharing one Krylov space.

TEST INFRASTRUCTURE ONLY, like the rest of this package: imported by tests/ and the CPU
baseline leg of the benchmark, never by the product library.

The paper solves D x = b with BiCGStab (Sec. 2) one right-hand side at a time.  For s
right-hand sides of the same matrix, the block variant of Guennouni, Jbilou and Sadok
("A block version of BiCGSTAB for linear systems with multiple right-hand sides",
Electronic Transactions on Numerical Analysis 16, 2003) replaces the scalars alpha and beta
by s x s matrices obtained from small linear solves against the shadow block R~0, and keeps
one scalar omega from Frobenius inner products.  With A = M_ee (even-odd Schur complement)
and B' the prepared right-hand sides (columns of n x s matrices):

    R = B' - A X,   R~ = R,   P = R
    repeat until every column j has |R_j| <= stop_j:
        V = A P
        alpha = (R~^H V)^-1 (R~^H R)                        s x s
        S = R - V alpha
        T = A S
        omega = <T, S>_F / <T, T>_F                         (0 when T = 0)
        X = X + P alpha + omega S
        R = S - omega T
        beta = -(R~^H V)^-1 (R~^H T)                        s x s
        P = R + (P - omega V) beta

For s = 1 this is the textbook BiCGStab: alpha = rho / <r~, v>, and since <r~, s> = 0 the
next rho equals -omega <r~, t>, so beta = -<r~, t> / <r~, v> = (rho'/rho)(alpha/omega).
The s x s solves use numpy.linalg.solve (LAPACK LU with partial pivoting) as a library step.
"""
import numpy as np

from . import (apply_Mee, apply_Mee_clov, clov_eo_prepare, clov_eo_reconstruct, eo_prepare, eo_reconstruct,
               parity_of_sites)


class BlockBreakdown(RuntimeError):
    """The s x s matrix R~^H V is singular to working precision or not finite.

    Singular to working precision means: a pivot of its LU factorisation with partial
    pivoting is at most 1e-13 times the largest entry.  The threshold comes from the
    backward error of that factorisation, not from any implementation: in FP64 (unit
    roundoff u = 2^-53 = 1.1e-16) LU of an s x s matrix is exact for a matrix within
    about s^2 u of it, relative to its largest entry, so for the block sizes used here
    (s <= 16: s^2 u = 2.8e-14) a pivot below a few times that bound cannot be told from
    zero, and 1e-13 (3.5 s^2 u at s = 16) is the smallest round threshold above it.  The
    pins separate the two regimes by many orders of magnitude either way: linearly
    dependent sources give relative pivots near u, independent random sources pivots of
    order 0.1 or more, so any threshold between about 1e-15 and 1e-3 classifies them alike."""


def _check_small(G):
    if not np.all(np.isfinite(G)):
        raise BlockBreakdown("non-finite block inner products")
    # LU pivots of G (partial pivoting), compared with the largest entry
    lu = G.copy()
    s = lu.shape[0]
    scale = np.abs(G).max()
    for k in range(s):
        p = k + int(np.argmax(np.abs(lu[k:, k])))
        lu[[k, p]] = lu[[p, k]]
        if not np.abs(lu[k, k]) > 1e-13 * scale:
            raise BlockBreakdown(f"pivot {k} of R~^H V is {abs(lu[k, k]):.3e} against {scale:.3e}")
        lu[k + 1:, k:] -= np.outer(lu[k + 1:, k] / lu[k, k], lu[k, k:])


def block_bicgstab(apply_A, Bp, stop, maxiter, X0=None):
    """The iteration above on n x s column blocks.  apply_A maps an n-vector to an n-vector;
    stop[j] is the absolute threshold of |R_j|.  Returns (X, iterations)."""
    n, s = Bp.shape
    A = lambda Y: np.stack([apply_A(Y[:, j]) for j in range(s)], axis=1)  # noqa: E731
    X = np.zeros_like(Bp) if X0 is None else X0.astype(np.complex128).copy()
    R = Bp - A(X) if X0 is not None else Bp.copy()
    Rt = R.copy()
    P = R.copy()
    it = 0
    while it < maxiter and not np.all(np.linalg.norm(R, axis=0) <= stop):
        V = A(P)
        G = Rt.conj().T @ V
        _check_small(G)
        alpha = np.linalg.solve(G, Rt.conj().T @ R)
        S = R - V @ alpha
        T = A(S)
        tt = np.vdot(T, T).real
        omega = np.vdot(T, S) / tt if tt > 0 else 0.0
        X = X + P @ alpha + omega * S
        R = S - omega * T
        beta = np.linalg.solve(G, -(Rt.conj().T @ T))
        P = R + (P - omega * V) @ beta
        it += 1
    return X, it


def solve_block(B, U, kappa, dims, tol, maxiter, F=None, X0=None):
    """Solve D x_j = b_j (D_clov with F) for the s right-hand sides B (s, V, 4, 3) together
    by block BiCGStab on M_ee.  tol: scalar or one per column; column j stops at
    |r_j| <= tol_j |b_j| (|b_j| of the full right-hand side, as for the single solver).
    X0 (optional): initial guesses (s, V, 4, 3), only their even sites are used.
    Returns (X (s, V, 4, 3), iterations, true relative residuals of the full system)."""
    from . import apply_D, apply_Dclov
    B = np.ascontiguousarray(B, np.complex128)
    s = B.shape[0]
    V = int(np.prod(dims))
    B = B.reshape(s, V, 4, 3)
    tol = np.broadcast_to(np.asarray(tol, np.float64), (s,))
    even = np.repeat(parity_of_sites(dims) == 0, 12)
    if F is None:
        prep = lambda b: eo_prepare(b, U, kappa, dims)  # noqa: E731
        A = lambda y: apply_Mee(y.reshape(V, 4, 3), U, kappa, dims).reshape(-1)  # noqa: E731
        rec = lambda xe, b: eo_reconstruct(xe, b, U, kappa, dims)  # noqa: E731
        full = lambda x: apply_D(x, U, kappa, dims)  # noqa: E731
    else:
        prep = lambda b: clov_eo_prepare(b, U, F, kappa, dims)  # noqa: E731
        A = lambda y: apply_Mee_clov(y.reshape(V, 4, 3), U, F, kappa, dims).reshape(-1)  # noqa: E731
        rec = lambda xe, b: clov_eo_reconstruct(xe, b, U, F, kappa, dims)  # noqa: E731
        full = lambda x: apply_Dclov(x, U, F, kappa, dims)  # noqa: E731
    Bp = np.stack([np.where(even, prep(B[j]).reshape(-1), 0) for j in range(s)], axis=1)
    bnorm = np.array([np.linalg.norm(B[j]) for j in range(s)])
    X0e = None
    if X0 is not None:
        X0 = np.asarray(X0, np.complex128).reshape(s, -1)
        X0e = np.stack([np.where(even, X0[j], 0) for j in range(s)], axis=1)
    Xe, it = block_bicgstab(A, Bp, tol * bnorm, maxiter, X0e)
    X = np.stack([rec(Xe[:, j].reshape(V, 4, 3), B[j]) for j in range(s)])
    res = np.array([np.linalg.norm(B[j] - full(X[j])) / bnorm[j] if bnorm[j] > 0 else 0.0 for j in range(s)])
    return X, it, res
