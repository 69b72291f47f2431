"""Seeded synthetic inputs: SU(3) gauge fields, clover terms and spinor sources.

This module holds input generators only, none of the Wilson operator's or the
solvers' arithmetic; both the GPU path and the CPU oracle are fed from it.

Gauge field (the paper generates no ensemble; a synthetic field stands in for a
Monte Carlo configuration):  for every site (x fastest) and direction mu (inner),
draw M with independent N(0,1) real and imaginary parts, form the Hermitian
H = (M + M^dag)/2, make it traceless, A = H - tr(H)/3, and set U = exp(i*eps*A).
det U = 1 and U is unitary to rounding.  eps = 0.3 gives <Re tr U>/3 ~ 0.89.

Random streams:  on the CPU the draws come from numpy's PCG64 (default_rng(seed)),
which is the canonical stream.  On a GPU device they come from torch's Philox
generator seeded with the same seed (fast for lattices with tens of millions of
links); the two streams differ, so a test that compares two sides always hands
both sides the same tensor.

Layouts (canonical, complex128): links (V, 4, 3, 3), spinors (V, 4, 3) or
(nrhs, V, 4, 3), site s = x + Lx*(y + Ly*(z + Lz*t)).
"""
import numpy as np
import torch


def volume(dims):
    return int(np.prod(dims))


def _gaussian_complex(shape, seed, device):
    if str(device) == "cpu":
        rng = np.random.default_rng(seed)
        a = rng.standard_normal(tuple(shape) + (2,))
        return torch.from_numpy(a[..., 0] + 1j * a[..., 1])
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    a = torch.randn(tuple(shape) + (2,), generator=g, device=device, dtype=torch.float64)
    return torch.complex(a[..., 0], a[..., 1])


def _traceless_hermitian(M):
    H = 0.5 * (M + M.conj().transpose(-1, -2))
    tr = torch.diagonal(H, dim1=-2, dim2=-1).sum(-1).real / 3.0
    eye = torch.eye(3, dtype=H.dtype, device=H.device)
    return H - tr[..., None, None] * eye


def su3_exp(A, eps):
    """U = exp(i*eps*A) for a batch of traceless Hermitian 3x3 A."""
    return torch.linalg.matrix_exp((1j * eps) * A)


def gauge_field(dims, eps=0.3, seed=1001, device="cpu", chunk=1 << 22):
    """Links U_mu(x) = exp(i*eps*A), shape (V, 4, 3, 3) complex128 on `device`."""
    V = volume(dims)
    M = _gaussian_complex((V, 4, 3, 3), seed, device)
    U = torch.empty((V, 4, 3, 3), dtype=torch.complex128, device=M.device)
    flatM = M.view(-1, 3, 3)
    flatU = U.view(-1, 3, 3)
    for i in range(0, flatM.shape[0], chunk):
        flatU[i:i + chunk] = su3_exp(_traceless_hermitian(flatM[i:i + chunk]), eps)
    del M
    return U


def unit_gauge(dims, device="cpu"):
    """Free field: every link is the 3x3 identity."""
    V = volume(dims)
    U = torch.zeros((V, 4, 3, 3), dtype=torch.complex128, device=device)
    U[..., 0, 0] = 1
    U[..., 1, 1] = 1
    U[..., 2, 2] = 1
    return U


def _gamma5_dirac():
    """gamma_5 of the Dirac basis used throughout (gamma_k = [[0,-i s_k],[i s_k,0]],
    gamma_4 = diag(1,1,-1,-1)): the 4x4 matrix -[[0,1],[1,0]] in 2x2 spin blocks."""
    g5 = np.zeros((4, 4))
    g5[0, 2] = g5[1, 3] = g5[2, 0] = g5[3, 1] = -1.0
    return g5


def clover_field(dims, c=0.05, seed=1201, device="cpu"):
    """Synthetic clover term F(x), shape (V, 12, 12) complex128 (rows and columns
    3*spin + colour, Dirac basis).  The paper builds F from the links and stores it
    like U without giving the construction; a stand-in with its structure is:
    F = c (P+ G1 P+ + P- G2 P-), P+- = (1 +- gamma_5)/2 (x) 1_colour, G1, G2 Hermitian
    with Gaussian entries (G = (M + M^dag)/2, M with N(0,1) real and imaginary parts),
    so F is Hermitian and commutes with gamma_5, i.e. block diagonal with two 6x6
    Hermitian blocks in the chiral basis.  c = 0.05 keeps |F| near 0.25."""
    V = volume(dims)
    M = _gaussian_complex((V, 2, 12, 12), seed, device)
    g5 = torch.from_numpy(np.kron(_gamma5_dirac(), np.eye(3))).to(M.device, torch.complex128)
    eye = torch.eye(12, dtype=torch.complex128, device=M.device)
    Pp, Pm = 0.5 * (eye + g5), 0.5 * (eye - g5)
    F = torch.empty((V, 12, 12), dtype=torch.complex128, device=M.device)
    chunk = 1 << 18
    for i in range(0, V, chunk):
        G = 0.5 * (M[i:i + chunk] + M[i:i + chunk].conj().transpose(-1, -2))
        F[i:i + chunk] = c * (Pp @ G[:, 0] @ Pp + Pm @ G[:, 1] @ Pm)
    del M
    return F


def random_su3(n, seed, eps=2.0, device="cpu"):
    """n random SU(3) matrices (for gauge transformations in tests)."""
    M = _gaussian_complex((n, 3, 3), seed, device)
    return su3_exp(_traceless_hermitian(M), eps)


def gaussian_source(dims, seed=2001, nrhs=None, device="cpu"):
    """Complex Gaussian spinor(s): re and im iid N(0,1); (V,4,3) or (nrhs,V,4,3)."""
    V = volume(dims)
    shape = (V, 4, 3) if nrhs is None else (nrhs, V, 4, 3)
    return _gaussian_complex(shape, seed, device)


def point_sources(dims, device="cpu"):
    """The 12 spin-colour point sources at the origin: rhs 3*spin + colour."""
    V = volume(dims)
    b = torch.zeros((12, V, 4, 3), dtype=torch.complex128, device=device)
    for s in range(4):
        for c in range(3):
            b[3 * s + c, 0, s, c] = 1.0
    return b
