"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle.

Tolerances:
  * FP64 Dslash: 1e-12 relative (norm-wise over the field) and every element within
    1e-12 of the field's largest element;
  * FP32 / FP16 Dslash: error against the FP64 oracle reported and bounded by the
    storage precision (FP32 5e-7, FP16 with per-site scales 2e-3, relative);
  * solves: the oracle's FP64 D applied to the GPU's x gives |b - D x| / |b| below the
    requested tolerance (every x with that residual is a correct answer); the distance
    to the oracle's own solution is reported and bounded by cond * tol.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1811_00893_amd import inputs

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
SHAPES = [(2, 2, 2, 2), (2, 4, 2, 6), (4, 4, 4, 4), (6, 4, 2, 6), (8, 8, 8, 8), (4, 6, 8, 10)]


@pytest.fixture(scope="module")
def L():
    from paper_1811_00893_amd import _lib
    return _lib


@pytest.fixture(scope="module")
def ctx(L):
    c = L.wilson_context_create()
    yield c
    L.wilson_context_destroy(c)


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def maxrel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def setup_case(dims, seed, eps=0.3):
    U = inputs.gauge_field(dims, eps=eps, seed=1000 + seed)
    psi = inputs.gaussian_source(dims, seed=2000 + seed)
    return U, psi


@pytest.mark.parametrize("dims", SHAPES)
def test_dslash_fp64_all_parities(L, ctx, dims):
    U, psi = setup_case(dims, 1)
    k = 0.125
    Un, pn = U.numpy(), psi.numpy()
    g = L.wilson_gauge_load(ctx, U.to(DEV), dims)
    try:
        for parity in (0, 1, 2):
            prev = inputs.gaussian_source(dims, seed=77)  # untouched sites must keep these values
            out = prev.to(DEV).clone()
            L.check(L.wilson_dslash_ex(ctx, g, out, psi.to(DEV), k, parity), "dslash_ex")
            torch.cuda.synchronize()
            ref = oracle.dslash(pn, Un, k, dims, parity, out=prev.numpy())
            got = out.cpu().numpy()
            print(f"dims={dims} parity={parity} rel={rel(got, ref):.2e} maxrel={maxrel(got, ref):.2e}")
            assert rel(got, ref) < 1e-12
            assert maxrel(got, ref) < 1e-12
            if parity < 2:
                par = oracle.parity_of_sites(dims)
                assert np.array_equal(got[par != parity], prev.numpy()[par != parity])
    finally:
        L.wilson_gauge_free(ctx, g)


def test_dslash_plain_entry_host_pointers(L):
    """wilson_dslash with host (numpy) buffers; out == in is allowed for a parity hop."""
    dims = (4, 2, 6, 4)
    U, psi = setup_case(dims, 2)
    Un, pn = U.numpy(), psi.numpy().copy()
    out = np.zeros_like(pn)
    assert L.wilson_dslash(out, pn, Un, 0.11, dims, 2) == 0
    assert rel(out, oracle.apply_D(pn, Un, 0.11, dims)) < 1e-12
    inplace = pn.copy()
    assert L.wilson_dslash(inplace, inplace, Un, 0.11, dims, 1) == 0
    ref = oracle.dslash(pn, Un, 0.11, dims, 1, out=pn)
    assert rel(inplace, ref) < 1e-12
    assert L.wilson_dslash(pn, pn, Un, 0.11, dims, 2) == L.WILSON_INVALID_ARG
    # the C ABI itself rejects an odd extent and a bad parity (raw symbol, no binding checks)
    bad = np.array([4, 2, 5, 4], np.int32)
    raw = L.lib().wilson_dslash
    assert raw(L._ptr(out), L._ptr(pn), L._ptr(Un), 0.11, bad.ctypes.data, 2) == L.WILSON_INVALID_ARG
    assert L.wilson_dslash(out, pn, Un, 0.11, dims, 3) == L.WILSON_INVALID_ARG
    assert raw(None, L._ptr(pn), L._ptr(Un), 0.11, np.array(dims, np.int32).ctypes.data, 0) == L.WILSON_INVALID_ARG


def test_dslash_kappa_zero_is_identity(L, ctx):
    dims = (4, 4, 2, 4)
    U, psi = setup_case(dims, 3)
    g = L.wilson_gauge_load(ctx, U.to(DEV), dims)
    out = torch.empty_like(psi, device=DEV)
    L.check(L.wilson_dslash_ex(ctx, g, out, psi.to(DEV), 0.0, 2), "dslash")
    assert torch.equal(out.cpu(), psi)
    L.wilson_gauge_free(ctx, g)


@pytest.mark.parametrize("prec,tol", [(1, 5e-7), (2, 2e-3), (3, 2e-3)])
def test_dslash_reduced_precision(L, ctx, prec, tol):
    dims = (8, 4, 6, 8)
    U, psi = setup_case(dims, 4)
    g = L.wilson_gauge_load(ctx, U.to(DEV), dims, L.WILSON_GAUGE_FP32 | L.WILSON_GAUGE_FP16)
    out = torch.empty_like(psi, device=DEV)
    L.check(L.wilson_dslash_ex(ctx, g, out, psi.to(DEV), 0.125, 2, prec), "dslash")
    ref = oracle.apply_D(psi.numpy(), U.numpy(), 0.125, dims)
    e = rel(out.cpu().numpy(), ref)
    print(f"precision {prec}: relative error vs FP64 oracle {e:.3e}")
    assert e < tol
    L.wilson_gauge_free(ctx, g)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_dslash_multi_rhs_matches_single(L, ctx, prec):
    dims = (4, 4, 4, 6)
    U, _ = setup_case(dims, 5)
    nrhs = 12
    psi = inputs.gaussian_source(dims, seed=99, nrhs=nrhs)
    g = L.wilson_gauge_load(ctx, U.to(DEV), dims, L.WILSON_GAUGE_FP32 | L.WILSON_GAUGE_FP16)
    out = torch.empty_like(psi, device=DEV)
    L.check(L.wilson_dslash_ex(ctx, g, out, psi.to(DEV), 0.12, 0, prec, nrhs), "dslash batch")
    par = oracle.parity_of_sites(dims)
    for k in (0, 5, 11):  # parity-0 hop: only even sites are written
        one = torch.zeros_like(psi[k], device=DEV)
        L.check(L.wilson_dslash_ex(ctx, g, one, psi[k].to(DEV).contiguous(), 0.12, 0, prec, 1), "dslash one")
        d = rel(out[k].cpu().numpy()[par == 0], one.cpu().numpy()[par == 0])
        print(f"prec {prec} rhs {k}: batched vs single {d:.2e}")
        assert d < (1e-6 if prec else 1e-14)
    ref = oracle.dslash(psi[3].numpy(), U.numpy(), 0.12, dims, 0)
    lim = {0: 1e-12, 1: 5e-7, 2: 2e-3}[prec]
    assert rel(out[3].cpu().numpy()[par == 0], ref[par == 0]) < lim
    L.wilson_gauge_free(ctx, g)


def oracle_residual(x, b, U, k, dims):
    r = b - oracle.apply_D(x, U, k, dims)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


@pytest.mark.parametrize("solver", [0, 1])
def test_solve_fp64_8x4(L, ctx, solver):
    """8^4, eps = 0.3, kappa = 0.12, tol 1e-10 (the small configuration)."""
    dims = (8, 8, 8, 8)
    k, tol = 0.12, 1e-10
    U = inputs.gauge_field(dims, eps=0.3, seed=1001)
    b = inputs.gaussian_source(dims, seed=2001)
    g = L.wilson_gauge_load(ctx, U.to(DEV), dims)
    x = torch.zeros_like(b, device=DEV)
    st, info = L.wilson_solve_ex(ctx, g, x, b.to(DEV), 1, k, tol, {"solver": solver, "maxiter": 5000})
    assert st == 0, (st, L.wilson_last_error(), info)
    xn = x.cpu().numpy()
    res = oracle_residual(xn, b.numpy(), U.numpy(), k, dims)
    xo, sto, tro = oracle.solve(b.numpy(), U.numpy(), k, dims, 1e-12, 5000, "bicgstab_eo")
    print(f"solver {solver}: iters {info[0]['iterations']} gpu true res {info[0]['true_residual']:.2e} "
          f"oracle-checked res {res:.2e}, |x - x_oracle|/|x_oracle| {rel(xn, xo):.2e}")
    assert res < tol
    assert abs(info[0]["true_residual"] - res) < 0.1 * tol
    assert rel(xn, xo) < 1e-6
    L.wilson_gauge_free(ctx, g)


def test_solve_plain_entry_and_lu(L):
    """wilson_solve on 2^4 equals the dense LU solve of Eq. (1) within cond * tol."""
    dims = (2, 2, 2, 2)
    U, b = setup_case(dims, 6)
    Un, bn = U.numpy(), b.numpy()
    x = np.zeros_like(bn)
    assert L.wilson_solve(x, bn, Un, 0.124, dims, 1e-12, 1000) == 0
    D = oracle.dense_D(Un, 0.124, dims)
    xl = np.linalg.solve(D, bn.ravel()).reshape(bn.shape)
    assert rel(x, xl) < 10 * np.linalg.cond(D) * 1e-12
    assert oracle_residual(x, bn, Un, 0.124, dims) < 1e-12


@pytest.mark.parametrize("prec", [1, 2, 3])
def test_solve_mixed_precision(L, ctx, prec):
    dims = (8, 8, 8, 8)
    k, tol = 0.125, 1e-10
    U = inputs.gauge_field(dims, eps=0.3, seed=1003)
    b = inputs.gaussian_source(dims, seed=2003)
    g = L.wilson_gauge_load(ctx, U.to(DEV), dims, L.WILSON_GAUGE_FP32 | L.WILSON_GAUGE_FP16)
    x = torch.zeros_like(b, device=DEV)
    st, info = L.wilson_solve_ex(ctx, g, x, b.to(DEV), 1, k, tol, {"precision": prec, "maxiter": 20000})
    assert st == 0, (st, L.wilson_last_error(), info)
    res = oracle_residual(x.cpu().numpy(), b.numpy(), U.numpy(), k, dims)
    print(f"precision {prec}: outer {info[0]['outer_cycles']} inner iters {info[0]['iterations']} res {res:.2e}")
    assert res < tol
    L.wilson_gauge_free(ctx, g)


def test_batched_point_sources(L, ctx):
    """12 point sources solved together equal the single-RHS solves; each passes the oracle."""
    dims = (4, 4, 4, 8)
    k, tol = 0.125, 1e-10
    U = inputs.gauge_field(dims, eps=0.3, seed=1004)
    b = inputs.point_sources(dims)
    g = L.wilson_gauge_load(ctx, U.to(DEV), dims, L.WILSON_GAUGE_FP32)
    for prec in (0, 1):
        x = torch.zeros_like(b, device=DEV)
        st, infos = L.wilson_solve_ex(ctx, g, x, b.to(DEV), 12, [k] * 12, [tol] * 12, {"precision": prec})
        assert st == 0, (st, L.wilson_last_error())
        xs = x.cpu().numpy()
        for j in (0, 4, 11):
            assert oracle_residual(xs[j], b[j].numpy(), U.numpy(), k, dims) < tol
            x1 = torch.zeros_like(b[j], device=DEV)
            st1, _ = L.wilson_solve_ex(ctx, g, x1, b[j].contiguous().to(DEV), 1, k, tol, {"precision": prec})
            assert st1 == 0
            d = rel(xs[j], x1.cpu().numpy())
            print(f"prec {prec} rhs {j}: batched vs single {d:.2e}")
            assert d < 1e-8
    L.wilson_gauge_free(ctx, g)


@pytest.mark.parametrize("cfg", ["256,1,1,0,0,1", "192,2,1,4,0,1", "128,3,1,0,0,1", "320,1,1,0,0,0,0,1",
                                 "256,1,1,4,0,1,1,0,1", "128,2,1,0,0,1,0,0,1",
                                 "256,1,1,0,0,1,1,0,1,2", "128,3,1,0,0,1,0,0,0,4", "64,2,1,0,0,0,0,0,0,1",
                                 "256,1,1,0,0,1,1,0,2", "128,2,1,0,0,1,0,0,2"])
def test_batched_solve_wave_split_configs(L, cfg, monkeypatch):
    """The batched solve with the hop's RHS groups split over the waves of a block (each
    wave writes its own partial sums of the fused reductions; also with the tile's links
    staged in LDS once for all waves), or with each block's directions split over its
    waves, converges for every RHS to the oracle's residual test (BiCGStab in FP64, FP32
    and with FP16 spinors, CGNR in FP64) and agrees with the default configuration."""
    dims = (4, 4, 8, 8)  # Vh = 512: eight 64-site tiles
    k, tol = 0.125, 1e-10
    U = inputs.gauge_field(dims, eps=0.3, seed=1005)
    b = inputs.point_sources(dims)
    ref = {}
    for forced in (False, True):
        if forced:
            monkeypatch.setenv("WILSON_HOP_CFG", cfg)
        c = L.wilson_context_create()
        g = L.wilson_gauge_load(c, U.to(DEV), dims, L.WILSON_GAUGE_FP32)
        try:
            # BiCGStab in FP64 and FP32, CGNR (gamma5 on the hops) in FP64, FP16 spinors
            for solver, prec in ((0, 0), (0, 1), (1, 0), (0, 3)):
                x = torch.zeros_like(b, device=DEV)
                st, _ = L.wilson_solve_ex(c, g, x, b.to(DEV), 12, [k] * 12, [tol] * 12,
                                          {"precision": prec, "solver": solver, "maxiter": 20000})
                assert st == 0, (cfg, solver, prec, st, L.wilson_last_error())
                xs = x.cpu().numpy()
                if not forced:
                    ref[solver, prec] = xs
                    continue
                for j in range(12):
                    assert oracle_residual(xs[j], b[j].numpy(), U.numpy(), k, dims) < tol, (cfg, solver, prec, j)
                d = rel(xs, ref[solver, prec])
                print(f"{cfg} solver {solver} prec {prec}: vs default {d:.2e}")
                assert d < 1e-7
        finally:
            L.wilson_gauge_free(c, g)
            L.wilson_context_destroy(c)


@pytest.mark.parametrize("cfg", ["256,1,1,0,0,0,1", "64,1,1,4,0,0,1", "320,1,1,0,0,0,0,1", "320,1,0,0,0,0,0,1",
                                 "256,1,1,0,0,0,1,0,0,2", "64,1,1,0,0,0,0,0,0,4"])
def test_solves_with_lane_exchange(L, cfg, monkeypatch):
    """Solves whose hops take x/y neighbours from other lanes, or split the eight
    directions over the waves of a block: BiCGStab and CGNR (gamma5 on the hop input and
    output) in FP64, and mixed precision with FP16 spinors, all to the oracle's residual
    test."""
    monkeypatch.setenv("WILSON_HOP_CFG", cfg)
    dims = (8, 8, 8, 8)
    k, tol = 0.125, 1e-10
    U = inputs.gauge_field(dims, eps=0.3, seed=1006)
    b = inputs.gaussian_source(dims, seed=2006)
    c = L.wilson_context_create()
    g = L.wilson_gauge_load(c, U.to(DEV), dims, L.WILSON_GAUGE_FP32 | L.WILSON_GAUGE_FP16)
    try:
        for solver, prec in ((0, 0), (1, 0), (0, 2), (0, 3)):
            x = torch.zeros_like(b, device=DEV)
            st, info = L.wilson_solve_ex(c, g, x, b.to(DEV), 1, k, tol,
                                         {"solver": solver, "precision": prec, "maxiter": 20000})
            assert st == 0, (cfg, solver, prec, st, L.wilson_last_error())
            res = oracle_residual(x.cpu().numpy(), b.numpy(), U.numpy(), k, dims)
            print(f"{cfg} solver {solver} prec {prec}: {info[0]['iterations']} iterations, residual {res:.2e}")
            assert res < tol
    finally:
        L.wilson_gauge_free(c, g)
        L.wilson_context_destroy(c)


def test_solve_edge_cases(L, ctx):
    dims = (4, 4, 2, 4)
    U, b = setup_case(dims, 8)
    g = L.wilson_gauge_load(ctx, U.to(DEV), dims)
    bd = b.to(DEV)
    # b = 0 -> x = 0
    x = torch.ones_like(bd)
    st, info = L.wilson_solve_ex(ctx, g, x, torch.zeros_like(bd), 1, 0.12, 1e-10)
    assert st == 0 and torch.count_nonzero(x) == 0
    # kappa = 0 -> x = b
    x = torch.zeros_like(bd)
    st, info = L.wilson_solve_ex(ctx, g, x, bd, 1, 0.0, 1e-12)
    assert st == 0 and rel(x.cpu().numpy(), b.numpy()) < 1e-14
    # maxiter = 1 -> not converged, x finite
    x = torch.zeros_like(bd)
    st, info = L.wilson_solve_ex(ctx, g, x, bd, 1, 0.125, 1e-12, {"maxiter": 1, "max_restarts": 0})
    assert st == L.WILSON_NOT_CONVERGED and torch.isfinite(x.real).all()
    # NaN in b
    bn = bd.clone()
    bn[3, 1, 2] = float("nan")
    st, _ = L.wilson_solve_ex(ctx, g, x, bn, 1, 0.12, 1e-10)
    assert st == L.WILSON_NONFINITE
    # invalid arguments
    assert L.wilson_solve_ex(ctx, g, x, bd, 1, -0.1, 1e-10)[0] == L.WILSON_INVALID_ARG
    assert L.wilson_solve_ex(ctx, g, x, bd, 1, 0.1, 0.0)[0] == L.WILSON_INVALID_ARG
    assert L.wilson_solve_ex(ctx, g, x, bd, 1, 0.1, 1e-10, {"maxiter": 0})[0] == L.WILSON_INVALID_ARG
    # initial guess: start from the solution -> converges at once
    x = torch.zeros_like(bd)
    assert L.wilson_solve_ex(ctx, g, x, bd, 1, 0.12, 1e-11)[0] == 0
    st, info = L.wilson_solve_ex(ctx, g, x, bd, 1, 0.12, 1e-10, {"use_x0": 1})
    assert st == 0 and info[0]["iterations"] == 0
    L.wilson_gauge_free(ctx, g)


def test_full_size_sampled_dslash(L, ctx):
    """32^3x64 (2.1M sites), FP64, in the launch configuration the benchmark times:
    2048 sampled sites of each parity against the oracle evaluated site by site."""
    dims = (32, 32, 32, 64)
    k = 0.125
    U = inputs.gauge_field(dims, eps=0.3, seed=1002, device=DEV)
    psi = inputs.gaussian_source(dims, seed=2002, device=DEV)
    g = L.wilson_gauge_load(ctx, U, dims)
    out = torch.empty_like(psi)
    L.check(L.wilson_dslash_ex(ctx, g, out, psi, k, 2), "dslash")
    torch.cuda.synchronize()
    Un, pn, on = U.cpu().numpy(), psi.cpu().numpy(), out.cpu().numpy()
    rng = np.random.default_rng(5)
    V = int(np.prod(dims))
    sites = np.concatenate([rng.choice(V, 4096, replace=False), [0, V - 1, 31, V - 32]])
    ref = pn[sites] - k * oracle.hop_sites(pn, Un, dims, sites)
    assert maxrel(on[sites], ref) < 1e-12
    L.wilson_gauge_free(ctx, g)
    del U, psi, out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("cfg", ["64,1,0,0", "128,1,1,0", "256,1,1,2", "64,1,1,4", "128,2,1,2", "64,4,1,2",
                                 "128,1,1,0,0,1", "256,1,1,2,0,1", "128,2,0,0,0,1", "256,1,1,0,40,1",
                                 "256,1,1,0,0,0,1", "64,1,1,4,0,0,1", "128,1,1,0,0,1,1", "256,1,1,2,0,0,1",
                                 "320,1,1,0,0,0,0,1", "320,1,0,0,0,0,0,1", "256,1,1,0,0,1,1,0,1",
                                 "128,2,1,2,0,1,0,0,1",
                                 # one z-plane per block of the visiting order (Lz/8 here: one
                                 # z-range per XCD), plain and with the wave split
                                 "64,1,1,1", "256,1,1,1,0,1,1,0,1",
                                 # t-marching over 5 or 1 slices of one t-parity: plain, two RHS per
                                 # lane, lane exchange, wave split with links in LDS, wave split
                                 # in plain block order, four RHS per lane (FP64: two)
                                 "64,1,1,0,0,0,0,0,0,5", "128,2,1,0,0,0,0,0,0,1", "64,1,1,0,0,0,1,0,0,5",
                                 "256,1,1,0,0,1,1,0,1,5", "128,1,0,0,0,1,0,0,0,1", "64,4,1,0,0,0,0,0,0,5",
                                 # links rebuilt to nine entries while staged in LDS (FP32 links;
                                 # FP64 falls back to the stored form)
                                 "256,1,1,0,0,1,1,0,2", "128,2,1,2,0,1,0,0,2"])
def test_dslash_every_launch_config(L, cfg, monkeypatch):
    """Every hop launch configuration the tuner can pick (block size, RHS per thread,
    XCD tile order, plane-blocked visiting order, LDS cap, RHS groups split over the
    waves of a block (with or without the tile's links staged in LDS), x/y neighbours
    exchanged between lanes, directions split over the waves of a block, blocks marching
    through t-slices) gives the oracle's result;
    the lattice has a ragged last block for every block size, rows of 3 sites (x wraps
    inside most wavefronts), with plane blocking wavefronts whose sites are not
    contiguous, and (t-marching) slices of 96 positions, so the last segment of each
    slice is ragged."""
    monkeypatch.setenv("WILSON_HOP_CFG", cfg)
    dims = (6, 4, 8, 10)  # Vh = 960: not a multiple of 64, 128 or 256
    U, _ = setup_case(dims, 9)
    nrhs = 4
    psi = inputs.gaussian_source(dims, seed=31, nrhs=nrhs)
    c = L.wilson_context_create()
    g = L.wilson_gauge_load(c, U.to(DEV), dims, L.WILSON_GAUGE_FP32 | L.WILSON_GAUGE_FP16)
    try:
        for prec, lim in ((0, 1e-12), (1, 5e-7), (2, 2e-3)):
            out = torch.zeros_like(psi, device=DEV)
            L.check(L.wilson_dslash_ex(c, g, out, psi.to(DEV), 0.125, 2, prec, nrhs), "dslash")
            for k in range(nrhs):
                ref = oracle.apply_D(psi[k].numpy(), U.numpy(), 0.125, dims)
                assert rel(out[k].cpu().numpy(), ref) < lim
    finally:
        L.wilson_gauge_free(c, g)
        L.wilson_context_destroy(c)


@pytest.mark.parametrize("prec", [0, 1, 3])
def test_solve_bitwise_reproducible(L, ctx, prec):
    """Reductions are summed in a fixed order on the device, so repeating a solve (after a
    first one has settled the tuned launch shapes) gives the same bits."""
    dims = (8, 4, 8, 8)
    U, b = setup_case(dims, 60)
    g = L.wilson_gauge_load(ctx, U.to(DEV), dims, L.WILSON_GAUGE_FP32 | L.WILSON_GAUGE_FP16)
    try:
        nrhs = 2
        bb = inputs.gaussian_source(dims, seed=2060, nrhs=nrhs).to(DEV)
        opts = {"precision": prec, "maxiter": 20000}
        xs, its = [], []
        for _ in range(3):
            x = torch.zeros_like(bb)
            st, info = L.wilson_solve_ex(ctx, g, x, bb, nrhs, [0.12, 0.125], [1e-10, 1e-11], opts)
            assert st == 0, L.wilson_last_error()
            xs.append(x.cpu())
            its.append([d["iterations"] for d in info])
        assert torch.equal(xs[1], xs[2]) and its[1] == its[2]
    finally:
        L.wilson_gauge_free(ctx, g)


def test_solve_info_counts_bytes_and_flops(L, ctx):
    """info.flops is 1320 operator flops per output site, right-hand side and hop launch;
    info.bytes is at least the hops' own algorithmic bytes (per output site in FP64: the
    8 links of 18 reals once for all right-hand sides, 24 reals in and 24 out per
    right-hand side) plus the 14 fused vector-field streams per BiCGStab iteration."""
    dims = (8, 8, 8, 8)
    U, b = setup_case(dims, 61)
    Vh = int(np.prod(dims)) // 2
    g = L.wilson_gauge_load(ctx, U.to(DEV), dims, 0)
    try:
        nrhs = 3
        bb = inputs.gaussian_source(dims, seed=2061, nrhs=nrhs).to(DEV)
        x = torch.zeros_like(bb)
        st, info = L.wilson_solve_ex(ctx, g, x, bb, nrhs, [0.12] * 3, [1e-10] * 3, {})
        assert st == 0
        d = info[0]
        assert all(e["flops"] == d["flops"] and e["bytes"] == d["bytes"] for e in info)
        assert d["flops"] == 1320.0 * Vh * nrhs * d["hop_launches"]
        it = max(e["iterations"] for e in info)
        low = d["hop_launches"] * Vh * (1152.0 + 384.0 * nrhs) + 14 * 192.0 * it * Vh * nrhs
        assert low <= d["bytes"] < 2.0 * low
    finally:
        L.wilson_gauge_free(ctx, g)


def test_maximum_rhs_count(L, ctx):
    """64 right-hand sides (the largest batch one call takes): the parity hop in FP64, FP32
    and FP16 against the oracle column by column, 65 rejected; the lockstep and the block
    solver (four blocks of 16) solve all 64 to tolerance by the oracle's D."""
    dims, k, n = (4, 4, 4, 8), 0.125, 64
    U = inputs.gauge_field(dims, eps=0.3, seed=2300)
    B = inputs.gaussian_source(dims, seed=2301, nrhs=n)
    g = L.wilson_gauge_load(ctx, U.to(DEV), dims, L.WILSON_GAUGE_FP32 | L.WILSON_GAUGE_FP16)
    try:
        Bd = B.to(DEV)
        for prec, limit in ((0, 1e-13), (1, 5e-7), (2, 2e-3)):
            out = torch.zeros_like(Bd)
            L.check(L.wilson_dslash_ex(ctx, g, out, Bd, k, 1, prec, n), "dslash")
            o = out.cpu().numpy()
            worst = max(rel(o[j], oracle.dslash(B[j].numpy(), U.numpy(), k, dims, 1)) for j in range(n))
            assert worst < limit, (prec, worst)
        big = inputs.gaussian_source(dims, seed=2302, nrhs=n + 1).to(DEV)
        assert L.wilson_dslash_ex(ctx, g, torch.zeros_like(big), big, k, 1, 0, n + 1) == L.WILSON_INVALID_ARG
        for solver in (L.WILSON_SOLVER_BICGSTAB_EO, L.WILSON_SOLVER_BLOCK_BICGSTAB_EO):
            x = torch.zeros_like(Bd)
            st, info = L.wilson_solve_ex(ctx, g, x, Bd, n, [k] * n, [1e-10] * n, {"solver": solver})
            assert st == 0, (solver, st, L.wilson_last_error())
            xn = x.cpu().numpy()
            worst = max(oracle_residual(xn[j], B[j].numpy(), U.numpy(), k, dims) for j in range(n))
            assert worst < 1e-10, (solver, worst)
    finally:
        L.wilson_gauge_free(ctx, g)
