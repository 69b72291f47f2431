"""GPU parity of the clover fermion matrix (D_clov = D_W + F, Sec. 2.1.2) against the FP64
oracle, through the C ABI.  Tolerances as for the Wilson matrix: FP64 1e-12 relative,
FP32 5e-7, FP16 spinors with per-site scales 2e-3; every solve passes the oracle's FP64
residual test with the clover matrix."""
import numpy as np
import pytest
import torch

import oracle
from paper_1811_00893_amd import inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def L():
    from paper_1811_00893_amd import _lib
    return _lib


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def maxrel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def clover_case(L, dims, seed, c=0.05):
    U = inputs.gauge_field(dims, seed=1300 + seed)
    F = inputs.clover_field(dims, c=c, seed=1400 + seed)
    ctx = L.wilson_context_create()
    g = L.wilson_gauge_load(ctx, U.to(DEV), dims, L.WILSON_GAUGE_FP32 | L.WILSON_GAUGE_FP16)
    assert L.wilson_gauge_attach_clover(ctx, g, F.to(DEV), dims) == 0, L.wilson_last_error()
    return U, F, ctx, g


def close(L, ctx, g):
    L.wilson_gauge_free(ctx, g)
    L.wilson_context_destroy(ctx)


def oracle_res(x, b, U, F, k, dims):
    return float(np.linalg.norm(b - oracle.apply_Dclov(x, U, F, k, dims)) / np.linalg.norm(b))


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 2, 6), (8, 8, 8, 8), (4, 6, 8, 10)])
def test_clover_dslash_all_precisions(L, dims):
    U, F, ctx, g = clover_case(L, dims, 1)
    try:
        k = 0.125
        psi = inputs.gaussian_source(dims, seed=1501)
        Un, Fn, pn = U.numpy(), F.numpy(), psi.numpy()
        ref = oracle.apply_Dclov(pn, Un, Fn, k, dims)
        for prec, lim in ((0, 1e-12), (1, 5e-7), (2, 2e-3), (3, 2e-3)):
            out = torch.zeros_like(psi, device=DEV)
            L.check(L.wilson_dslash_ex(ctx, g, out, psi.to(DEV), k, 2, prec, 1), "dslash")
            o = out.cpu().numpy()
            print(f"{dims} precision {prec}: rel {rel(o, ref):.2e}")
            assert rel(o, ref) < lim and maxrel(o, ref) < 10 * lim
        # the parity blocks are the off-diagonal -kappa H, the same as for the Wilson matrix
        for par in (0, 1):
            out = torch.zeros_like(psi, device=DEV)
            L.check(L.wilson_dslash_ex(ctx, g, out, psi.to(DEV), k, par, 0, 1), "dslash")
            r = oracle.dslash(pn, Un, k, dims, par)
            assert rel(out.cpu().numpy(), r) < 1e-12
    finally:
        close(L, ctx, g)


def test_clover_dslash_multi_rhs(L):
    dims = (8, 4, 4, 8)
    U, F, ctx, g = clover_case(L, dims, 2)
    try:
        k = 0.12
        nrhs = 4
        psi = inputs.gaussian_source(dims, seed=1502, nrhs=nrhs)
        for prec, lim in ((0, 1e-12), (1, 5e-7)):
            out = torch.zeros_like(psi, device=DEV)
            L.check(L.wilson_dslash_ex(ctx, g, out, psi.to(DEV), k, 2, prec, nrhs), "dslash")
            for j in range(nrhs):
                ref = oracle.apply_Dclov(psi[j].numpy(), U.numpy(), F.numpy(), k, dims)
                assert rel(out[j].cpu().numpy(), ref) < lim
    finally:
        close(L, ctx, g)


def test_clover_zero_equals_wilson_and_detach(L):
    dims = (4, 4, 4, 8)
    U = inputs.gauge_field(dims, seed=1310)
    psi = inputs.gaussian_source(dims, seed=1510)
    ctx = L.wilson_context_create()
    g = L.wilson_gauge_load(ctx, U.to(DEV), dims, L.WILSON_GAUGE_FP32)
    try:
        wil = torch.zeros_like(psi, device=DEV)
        L.check(L.wilson_dslash_ex(ctx, g, wil, psi.to(DEV), 0.13, 2, 0, 1), "dslash")
        bytes0 = L.wilson_gauge_bytes(g)
        Fz = torch.zeros((int(np.prod(dims)), 12, 12), dtype=torch.complex128)
        assert L.wilson_gauge_attach_clover(ctx, g, Fz.to(DEV), dims) == 0
        assert L.wilson_gauge_bytes(g) >= bytes0 + 1728 * int(np.prod(dims))
        clv = torch.zeros_like(psi, device=DEV)
        L.check(L.wilson_dslash_ex(ctx, g, clv, psi.to(DEV), 0.13, 2, 0, 1), "dslash")
        assert rel(clv.cpu().numpy(), wil.cpu().numpy()) < 1e-15
        L.wilson_gauge_detach_clover(ctx, g)
        assert L.wilson_gauge_bytes(g) == bytes0
        again = torch.zeros_like(psi, device=DEV)
        L.check(L.wilson_dslash_ex(ctx, g, again, psi.to(DEV), 0.13, 2, 0, 1), "dslash")
        assert torch.equal(again, wil)
    finally:
        close(L, ctx, g)


@pytest.mark.parametrize("solver,prec", [(0, 0), (1, 0), (0, 1), (0, 2), (0, 3), (1, 1)])
def test_clover_solves(L, solver, prec):
    dims = (8, 8, 8, 8)
    k, tol = 0.125, 1e-10
    U, F, ctx, g = clover_case(L, dims, 3)
    try:
        b = inputs.gaussian_source(dims, seed=1503)
        x = torch.zeros_like(b, device=DEV)
        st, info = L.wilson_solve_ex(ctx, g, x, b.to(DEV), 1, k, tol,
                                     {"solver": solver, "precision": prec, "maxiter": 20000})
        assert st == 0, (st, L.wilson_last_error(), info)
        res = oracle_res(x.cpu().numpy(), b.numpy(), U.numpy(), F.numpy(), k, dims)
        xo, sto, tro = oracle.solve_clov(b.numpy(), U.numpy(), F.numpy(), k, dims, 1e-12, 20000, "bicgstab_eo")
        d = rel(x.cpu().numpy(), xo)
        print(f"solver {solver} precision {prec}: {info[0]['iterations']} iterations, "
              f"{info[0]['outer_cycles']} outer, residual {res:.2e}, vs oracle solution {d:.2e}")
        assert res < tol
        assert d < 1e-7
    finally:
        close(L, ctx, g)


def test_clover_batched_solve_and_batch_api(L):
    """Several right-hand sides in one solve, and one through the serving batch API, each
    to the oracle's clover residual test."""
    dims = (4, 4, 8, 8)
    k, tol = 0.12, 1e-10
    U, F, ctx, g = clover_case(L, dims, 4)
    try:
        nrhs = 3
        b = inputs.gaussian_source(dims, seed=1504, nrhs=nrhs)
        for prec in (0, 1):
            x = torch.zeros_like(b, device=DEV)
            st, _ = L.wilson_solve_ex(ctx, g, x, b.to(DEV), nrhs, [k] * nrhs, [tol] * nrhs, {"precision": prec})
            assert st == 0, L.wilson_last_error()
            for j in range(nrhs):
                assert oracle_res(x[j].cpu().numpy(), b[j].numpy(), U.numpy(), F.numpy(), k, dims) < tol
        bat = L.wilson_batch_create(ctx, g, 2, {"precision": 1})
        b0 = b[0].contiguous().to(DEV)
        assert L.wilson_batch_attach(bat, 1, b0, k, tol) == 0
        for _ in range(500):
            L.wilson_batch_step(bat, 4)
            state, status = L.wilson_batch_poll(bat, 2)
            if state[1] == 2:
                break
        x = torch.zeros_like(b0)
        st, info = L.wilson_batch_detach(bat, 1, x)
        assert st == 0 and info["converged"] == 1
        assert oracle_res(x.cpu().numpy(), b[0].numpy(), U.numpy(), F.numpy(), k, dims) < tol
        L.wilson_batch_destroy(bat)
    finally:
        close(L, ctx, g)


def test_clover_attach_rejects_bad_terms(L):
    dims = (4, 4, 4, 4)
    V = int(np.prod(dims))
    U = inputs.gauge_field(dims, seed=1320)
    ctx = L.wilson_context_create()
    g = L.wilson_gauge_load(ctx, U.to(DEV), dims)
    try:
        F = inputs.clover_field(dims, seed=1420)
        bad = F.clone()
        bad[3, 0, 1] += 0.01  # no longer Hermitian
        assert L.wilson_gauge_attach_clover(ctx, g, bad.to(DEV), dims) == L.WILSON_INVALID_ARG
        cpl = F.clone()
        # commuting with gamma5 = -[[0,1],[1,0]] needs F_uu = F_ll and F_ul = F_lu on the spin
        # pairs; a real change of one upper diagonal entry keeps F Hermitian and breaks that
        cpl[5, 0, 0] += 0.01
        assert L.wilson_gauge_attach_clover(ctx, g, cpl.to(DEV), dims) == L.WILSON_INVALID_ARG
        sing = torch.zeros((V, 12, 12), dtype=torch.complex128)
        sing[7] = -torch.eye(12, dtype=torch.complex128)  # T = 1 + F = 0 at site 7
        assert L.wilson_gauge_attach_clover(ctx, g, sing.to(DEV), dims) == L.WILSON_INVALID_ARG
        assert L.wilson_gauge_bytes(g) < 1728 * V  # nothing was attached
        assert L.wilson_gauge_attach_clover(ctx, g, F.to(DEV), dims) == 0  # host array too
        assert L.wilson_gauge_attach_clover(ctx, g, F, dims) == 0
    finally:
        close(L, ctx, g)


@pytest.mark.parametrize("cfg", ["64,2,1,4", "128,1,1,0,0,1", "256,1,0,0,40,0,1", "320,1,1,0,0,0,0,1"])
def test_clover_every_launch_config(L, cfg, monkeypatch):
    """Pinned launch configurations are fitted to the clover kernels (one RHS per lane,
    no lane exchange) and give the oracle's D_clov."""
    monkeypatch.setenv("WILSON_HOP_CFG", cfg)
    dims = (6, 4, 8, 10)
    U, F, ctx, g = clover_case(L, dims, 5)
    try:
        nrhs = 4
        psi = inputs.gaussian_source(dims, seed=1505, nrhs=nrhs)
        out = torch.zeros_like(psi, device=DEV)
        L.check(L.wilson_dslash_ex(ctx, g, out, psi.to(DEV), 0.125, 2, 0, nrhs), "dslash")
        for j in range(nrhs):
            ref = oracle.apply_Dclov(psi[j].numpy(), U.numpy(), F.numpy(), 0.125, dims)
            assert rel(out[j].cpu().numpy(), ref) < 1e-12
    finally:
        close(L, ctx, g)
