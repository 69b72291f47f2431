"""On small lattices the BiCGStab iteration lets the vector kernel after each of its two
reducing hops (the s update, the x/r update) run that hop's finalize (alpha, omega) before
its own work, instead of a finalize kernel of its own: every block sums the hop's partials
in the finalize kernel's order and with its arithmetic, so every solution must be bitwise
the one with separate finalize kernels (WILSON_FUSE_FIN=0), for BiCGStab and CGNR, FP64
and mixed precision (FP32 and FP16 inner fields), several right-hand sides, and the batch
engine; each solution also passes the oracle's residual check."""
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


@pytest.mark.parametrize("dims,opts,nrhs", [
    ((8, 8, 8, 8), {"precision": 0}, 1),
    ((8, 8, 8, 8), {"precision": 0, "solver": 1}, 2),
    ((8, 8, 8, 8), {"precision": 1}, 3),
    ((4, 4, 8, 8), {"precision": 3}, 2),
    ((4, 4, 4, 8), {"precision": 2, "solver": 1}, 1),
    ((16, 16, 16, 32), {"precision": 1}, 1),
], ids=["8^4_bicgstab_fp64", "8^4_cgnr_fp64_2rhs", "8^4_mixed_fp32_3rhs", "4^2x8^2_fp16_2rhs",
        "4^3x8_fp16_fp32links_cgnr", "16^3x32_mixed_fp32"])
def test_fused_finalize_is_bitwise_the_finalize_kernel(L, dims, opts, nrhs, monkeypatch):
    print(f"fused finalize {dims} {opts} nrhs {nrhs}", flush=True)
    k, tol = 0.12, 1e-10
    U = inputs.gauge_field(dims, eps=0.3, seed=1801)
    b = inputs.gaussian_source(dims, seed=1802, nrhs=nrhs).to(DEV)
    kap = [k + 0.001 * j for j in range(nrhs)]
    results = {}
    for fuse in ("0", "1"):
        monkeypatch.setenv("WILSON_FUSE_FIN", fuse)
        ctx = L.wilson_context_create()
        g = L.wilson_gauge_load(ctx, U.to(DEV), dims, L.WILSON_GAUGE_FP32 | L.WILSON_GAUGE_FP16)
        try:
            xs = []
            for _ in range(2):
                x = torch.zeros_like(b)
                st, info = L.wilson_solve_ex(ctx, g, x, b, nrhs, kap, tol, opts)
                assert st == 0, L.wilson_last_error()
                xs.append((x.clone(), [i["iterations"] for i in info], [i["true_residual"] for i in info]))
            results[fuse] = xs
        finally:
            L.wilson_gauge_free(ctx, g)
            L.wilson_context_destroy(ctx)
    for (xa, ia, ra), (xb, ib, rb) in zip(results["0"], results["1"]):
        assert ia == ib
        assert ra == rb
        assert torch.equal(xa, xb)
    xn, bn = results["1"][0][0].cpu().numpy(), b.cpu().numpy()
    for j in range(nrhs):
        assert residual(xn[j], bn[j], U.numpy(), kap[j], dims) < tol


def test_fused_finalize_in_the_batch_engine(L, monkeypatch):
    """Requests attached to a batch at different times (slots at different iterations)."""
    dims = (8, 8, 8, 8)
    U = inputs.gauge_field(dims, eps=0.3, seed=1803)
    srcs = [inputs.gaussian_source(dims, seed=1804 + j).to(DEV) for j in range(3)]
    results = {}
    for fuse in ("0", "1"):
        monkeypatch.setenv("WILSON_FUSE_FIN", fuse)
        ctx = L.wilson_context_create()
        g = L.wilson_gauge_load(ctx, U.to(DEV), dims, L.WILSON_GAUGE_FP32)
        bat = L.wilson_batch_create(ctx, g, 4, {"precision": 1})
        try:
            xs = {}
            attached = 0
            for step in range(500):
                if attached < 3 and step % 3 == 0:
                    assert L.wilson_batch_attach(bat, attached, srcs[attached], 0.12 + 0.002 * attached, 1e-10) == 0
                    attached += 1
                L.wilson_batch_step(bat, 2)
                state, status = L.wilson_batch_poll(bat, 4)
                for j in range(attached):
                    if state[j] == 2 and j not in xs:
                        assert status[j] == 0
                        x = torch.zeros_like(srcs[j])
                        assert L.wilson_batch_detach(bat, j, x)[0] == 0
                        xs[j] = x
                if len(xs) == 3:
                    break
            assert len(xs) == 3
            results[fuse] = xs
        finally:
            L.wilson_batch_destroy(bat)
            L.wilson_gauge_free(ctx, g)
            L.wilson_context_destroy(ctx)
    for j in range(3):
        assert torch.equal(results["0"][j], results["1"][j])
        r = residual(results["1"][j].cpu().numpy(), srcs[j].cpu().numpy(), U.numpy(), 0.12 + 0.002 * j, dims)
        assert r < 1e-10
