"""Small lattices replay chunks of solver iterations from captured HIP graphs (kernel nodes
only).  The graphs run the kernels of the ordinary path with the same arguments, so every
solution must be bitwise the one the ordinary path gives (WILSON_GRAPHS=0), for BiCGStab
and CGNR, in FP64 and mixed precision, with several right-hand sides; each solve replays
its graphs many times, and the solves run back to back with eager work and
synchronisations in between.  Every solution also passes the oracle's residual check."""
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


def residual(x, b, U, k, dims):
    return float(np.linalg.norm(b - oracle.apply_D(x, U, k, dims)) / np.linalg.norm(b))


@pytest.mark.parametrize("dims,opts", [
    ((8, 8, 8, 8), {"precision": 0}),
    ((8, 8, 8, 8), {"precision": 0, "solver": 1}),
    ((8, 8, 8, 8), {"precision": 1}),
    ((4, 4, 8, 8), {"precision": 3}),
    ((16, 16, 16, 32), {"precision": 0}),
], ids=["8^4_bicgstab_fp64", "8^4_cgnr_fp64", "8^4_mixed_fp32", "4^2x8^2_mixed_fp16", "16^3x32_fp64"])
def test_graph_replay_is_bitwise_the_ordinary_path(L, dims, opts, monkeypatch):
    k, tol, nrhs = 0.12, 1e-10, 3
    U = inputs.gauge_field(dims, eps=0.3, seed=1701)
    b = inputs.gaussian_source(dims, seed=1702, nrhs=nrhs).to(DEV)
    results = {}
    for graphs in ("0", "1"):
        monkeypatch.setenv("WILSON_GRAPHS", graphs)
        ctx = L.wilson_context_create()
        g = L.wilson_gauge_load(ctx, U.to(DEV), dims, L.WILSON_GAUGE_FP32 | L.WILSON_GAUGE_FP16)
        try:
            xs = []
            for rep in range(3):
                x = torch.zeros_like(b)
                st, info = L.wilson_solve_ex(ctx, g, x, b, nrhs, [k + 0.001 * j for j in range(nrhs)], tol, opts)
                assert st == 0, L.wilson_last_error()
                torch.cuda.synchronize()
                xs.append((x.clone(), [i["iterations"] for i in info]))
                b.mul_(1.0)  # eager work between the solves
                torch.cuda.synchronize()
            results[graphs] = xs
        finally:
            L.wilson_gauge_free(ctx, g)
            L.wilson_context_destroy(ctx)
    for (xa, ia), (xb, ib) in zip(results["0"], results["1"]):
        assert ia == ib
        assert torch.equal(xa, xb)
    xn, bn = results["1"][-1][0].cpu().numpy(), b.cpu().numpy()
    for j in range(nrhs):
        assert residual(xn[j], bn[j], U.numpy(), k + 0.001 * j, dims) < tol


def test_graph_replay_follows_the_bound_gauge_field(L, monkeypatch):
    """One context solves on two gauge fields of the same shape in turn: its cached solve
    workspace is bound to each in turn, and a chunk captured on one field must not be
    replayed on the other."""
    dims, k, tol = (8, 8, 8, 8), 0.12, 1e-10
    Us = [inputs.gauge_field(dims, eps=e, seed=s) for e, s in ((0.3, 1711), (0.2, 1712))]
    b = inputs.gaussian_source(dims, seed=1713).to(DEV)
    results = {}
    for graphs in ("0", "1"):
        monkeypatch.setenv("WILSON_GRAPHS", graphs)
        ctx = L.wilson_context_create()
        gs = [L.wilson_gauge_load(ctx, U.to(DEV), dims) for U in Us]
        try:
            xs = []
            for rep in range(4):
                x = torch.zeros_like(b)
                st, _ = L.wilson_solve_ex(ctx, gs[rep % 2], x, b, 1, k, tol)
                assert st == 0, L.wilson_last_error()
                xs.append(x.clone())
            results[graphs] = xs
        finally:
            for g in gs:
                L.wilson_gauge_free(ctx, g)
            L.wilson_context_destroy(ctx)
    for xa, xb in zip(results["0"], results["1"]):
        assert torch.equal(xa, xb)
    for rep, x in enumerate(results["1"]):
        U = Us[rep % 2]
        assert residual(x.cpu().numpy(), b.cpu().numpy(), U.numpy(), k, dims) < tol
