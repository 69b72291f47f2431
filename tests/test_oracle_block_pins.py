"""Pins of the oracle's block BiCGStab (several right-hand sides sharing one Krylov space)
against facts that do not come from the block code itself:
  * one right-hand side: the block recurrence is the textbook BiCGStab, so its iterates
    equal those of the oracle's C BiCGStab (written with the other beta formula,
    (rho'/rho)(alpha/omega)) at every fixed iteration count;
  * finite termination: the block Krylov space of s columns fills the n-dimensional even
    space after n/s steps, so on 2^4 (n = 96 even unknowns) 12 columns converge in 8 steps,
    where one column is still far off;
  * right-multiplying the sources by a unitary s x s matrix Q multiplies every iterate by Q
    (a transposed or conjugated alpha or beta, or a product on the wrong side, breaks it);
  * converged columns solve the full system, checked with the oracle's D and D_clov;
  * linearly dependent right-hand sides make R~^H V singular and are reported.
"""
import numpy as np
import pytest

from paper_1811_00893_amd import inputs


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def test_one_column_is_bicgstab(oracle_mod):
    dims, k = (4, 4, 4, 8), 0.125
    U = inputs.gauge_field(dims, eps=0.3, seed=2100).numpy()
    b = inputs.gaussian_source(dims, seed=2101).numpy()
    for it in (1, 2, 5, 9):
        x_ref, st, _ = oracle_mod.solve(b, U, k, dims, 0.0, it, "bicgstab_eo")
        X, n, _ = oracle_mod.solve_block(b[None], U, k, dims, 0.0, it)
        assert n == it and st == -1
        assert rel(X[0], x_ref) < 1e-13, it


def test_finite_termination_on_2x2x2x2(oracle_mod):
    dims, k = (2, 2, 2, 2), 0.15
    U = inputs.gauge_field(dims, eps=0.5, seed=2110).numpy()
    B = inputs.gaussian_source(dims, seed=2111, nrhs=12).numpy()
    _, _, res7 = oracle_mod.solve_block(B, U, k, dims, 0.0, 7)
    _, _, res8 = oracle_mod.solve_block(B, U, k, dims, 0.0, 8)
    _, _, res1 = oracle_mod.solve_block(B[:1], U, k, dims, 0.0, 8)
    assert res7.max() > 1e-10
    assert res8.max() < 1e-12
    assert res1.max() > 1e-7


def test_unitary_change_of_sources(oracle_mod):
    dims, k, s = (4, 4, 4, 8), 0.125, 4
    U = inputs.gauge_field(dims, eps=0.3, seed=2120).numpy()
    B = inputs.gaussian_source(dims, seed=2121, nrhs=s).numpy()
    rng = np.random.default_rng(2122)
    Q, _ = np.linalg.qr(rng.normal(size=(s, s)) + 1j * rng.normal(size=(s, s)))
    mix = lambda Y: np.tensordot(Q, Y, axes=([0], [0]))  # noqa: E731  (Y Q column-wise: sum_j Q[j,k] Y_j)
    for it in (1, 4):
        X, _, _ = oracle_mod.solve_block(B, U, k, dims, 0.0, it)
        XQ, _, _ = oracle_mod.solve_block(mix(B), U, k, dims, 0.0, it)
        assert rel(XQ, mix(X)) < 1e-13, it
    # a non-unitary mix is not an invariance of the Frobenius omega
    C = Q * np.array([1.0, 3.0, 0.2, 1.0])
    XC, _, _ = oracle_mod.solve_block(np.tensordot(C, B, axes=([0], [0])), U, k, dims, 0.0, 4)
    assert rel(XC, np.tensordot(C, X, axes=([0], [0]))) > 1e-8


@pytest.mark.parametrize("clover", [False, True])
def test_converged_columns_solve_the_full_system(oracle_mod, clover):
    dims, k = (4, 4, 4, 8), 0.125
    U = inputs.gauge_field(dims, eps=0.3, seed=2130).numpy()
    B = inputs.point_sources(dims).numpy()[:6]
    F = inputs.clover_field(dims, c=0.05, seed=2131).numpy() if clover else None
    tol = [1e-8, 1e-10, 1e-9, 1e-10, 1e-11, 1e-10]
    X, n, res = oracle_mod.solve_block(B, U, k, dims, tol, 500, F=F)
    assert 0 < n < 500
    for j in range(6):
        r = B[j] - (oracle_mod.apply_Dclov(X[j], U, F, k, dims) if clover else oracle_mod.apply_D(X[j], U, k, dims))
        assert np.linalg.norm(r) / np.linalg.norm(B[j]) < tol[j]
        assert abs(res[j] - np.linalg.norm(r) / np.linalg.norm(B[j])) < 1e-14


def test_dependent_sources_break_down(oracle_mod):
    dims = (4, 4, 4, 4)
    U = inputs.gauge_field(dims, seed=2140).numpy()
    b = inputs.gaussian_source(dims, seed=2141, nrhs=2).numpy()
    B = np.stack([b[0], b[1], 2.0 * b[0] - 1j * b[1]])
    with pytest.raises(oracle_mod.BlockBreakdown):
        oracle_mod.solve_block(B, U, 0.12, dims, 1e-10, 100)


def test_breakdown_threshold_separates_dependent_sources(oracle_mod):
    """The breakdown test (a relative LU pivot of R~^H V at most 1e-13) sits far from both
    regimes: on the first iteration, linearly dependent sources give a smallest relative
    pivot near the unit roundoff, independent Gaussian or point sources pivots of order one
    (LU from scipy, independent of the oracle's own pivot loop)."""
    import scipy.linalg
    dims = (4, 4, 4, 4)
    V = int(np.prod(dims))
    U = inputs.gauge_field(dims, seed=2140).numpy()
    even = np.repeat(oracle_mod.parity_of_sites(dims) == 0, 12)

    def min_pivot(B):
        Bp = np.stack([np.where(even, oracle_mod.eo_prepare(B[j], U, 0.12, dims).reshape(-1), 0)
                       for j in range(B.shape[0])], axis=1)
        AV = np.stack([oracle_mod.apply_Mee(Bp[:, j].reshape(V, 4, 3), U, 0.12, dims).reshape(-1)
                       for j in range(Bp.shape[1])], axis=1)
        G = Bp.conj().T @ AV
        _, _, u = scipy.linalg.lu(G)
        return float(np.abs(np.diag(u)).min() / np.abs(G).max())

    b = inputs.gaussian_source(dims, seed=2141, nrhs=12).numpy()
    assert min_pivot(np.stack([b[0], b[1], 2.0 * b[0] - 1j * b[1]])) < 1e-15
    assert min_pivot(b) > 1e-3
    assert min_pivot(inputs.point_sources(dims).numpy()) > 1e-3
