"""Independent restatements used to pin the oracle (test helpers, numpy only).

Nothing here calls the oracle; each function builds its object a different way
from the oracle's site loop:
  * gamma matrices as Kronecker products of Pauli matrices (Dirac basis);
  * D assembled as a dense matrix block by block from Eq. (1) of Sec. 2.1;
  * the free-field momentum-space operator and its FFT inverse (closed form).
"""
import numpy as np

SIG = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]], complex),
       np.array([[1, 0], [0, -1]], complex)]
I2 = np.eye(2, dtype=complex)


def gammas():
    """Dirac basis: gamma_k = sigma_y (x) sigma_k (k = x,y,z), gamma_t = sigma_z (x) 1, gamma_5 = g1 g2 g3 g4."""
    g = [np.kron(SIG[1], SIG[k]) for k in range(3)] + [np.kron(SIG[2], I2)]
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    return g, g5


def coords(dims):
    """(V, 4) array of (x, y, z, t) with x fastest."""
    Lx, Ly, Lz, Lt = dims
    t, z, y, x = np.unravel_index(np.arange(Lx * Ly * Lz * Lt), (Lt, Lz, Ly, Lx))
    return np.stack([x, y, z, t], axis=1)


def site_of(c, dims):
    Lx, Ly, Lz, Lt = dims
    return c[..., 0] + Lx * (c[..., 1] + Ly * (c[..., 2] + Lz * c[..., 3]))


def dense_wilson(U, kappa, dims):
    """Dense D = 1 - kappa*sum_mu[(1-g_mu)(x)U_mu(x) d_{x+mu,y} + (1+g_mu)(x)U_mu(x-mu)^dag d_{x-mu,y}],
    antiperiodic in t (sign -1 on hops across the t wrap), periodic otherwise."""
    dims = tuple(int(d) for d in dims)
    V = int(np.prod(dims))
    U = np.asarray(U).reshape(V, 4, 3, 3)
    g, _ = gammas()
    one = np.eye(4, dtype=complex)
    D = np.eye(12 * V, dtype=complex)
    C = coords(dims)
    for s in range(V):
        for mu in range(4):
            cf = C[s].copy(); cf[mu] = (cf[mu] + 1) % dims[mu]
            cb = C[s].copy(); cb[mu] = (cb[mu] - 1) % dims[mu]
            sf, sb = site_of(cf, dims), site_of(cb, dims)
            sgn_f = -1.0 if (mu == 3 and C[s][3] == dims[3] - 1) else 1.0
            sgn_b = -1.0 if (mu == 3 and C[s][3] == 0) else 1.0
            D[12 * s:12 * s + 12, 12 * sf:12 * sf + 12] -= kappa * sgn_f * np.kron(one - g[mu], U[s, mu])
            D[12 * s:12 * s + 12, 12 * sb:12 * sb + 12] -= kappa * sgn_b * np.kron(one + g[mu], U[sb, mu].conj().T)
    return D


def parity(dims):
    c = coords(dims)
    return c.sum(axis=1) & 1


def free_field_momentum_op(p, kappa):
    """D(p) = (1 - 2k sum cos p_mu) 1 + 2ik sum sin p_mu gamma_mu (4x4), from Eq. (1) with U = 1."""
    g, _ = gammas()
    A = 1 - 2 * kappa * np.sum(np.cos(p))
    M = A * np.eye(4, dtype=complex)
    for mu in range(4):
        M = M + 2j * kappa * np.sin(p[mu]) * g[mu]
    return M


def free_field_solve_fft(b, kappa, dims):
    """x = D^{-1} b for U = 1 in momentum space.  The antiperiodic t boundary is removed
    by the twist b -> exp(-i pi t / Lt) b, which makes the problem periodic in t with
    the momentum shifted by pi/Lt."""
    Lx, Ly, Lz, Lt = dims
    b = np.asarray(b).reshape(Lt, Lz, Ly, Lx, 4, 3)
    t = np.arange(Lt)[:, None, None, None, None, None]
    tw = np.exp(-1j * np.pi * t / Lt)
    bt = np.fft.fftn(b * tw, axes=(0, 1, 2, 3))
    g, _ = gammas()
    pt = 2 * np.pi * np.fft.fftfreq(Lt) * 1.0 + np.pi / Lt
    pz = 2 * np.pi * np.fft.fftfreq(Lz)
    py = 2 * np.pi * np.fft.fftfreq(Ly)
    px = 2 * np.pi * np.fft.fftfreq(Lx)
    PT, PZ, PY, PX = np.meshgrid(pt, pz, py, px, indexing="ij")
    P = [PX, PY, PZ, PT]
    A = 1 - 2 * kappa * (np.cos(PX) + np.cos(PY) + np.cos(PZ) + np.cos(PT))
    B = [2 * kappa * np.sin(q) for q in P]
    den = A ** 2 + sum(bb ** 2 for bb in B)
    # D(p)^{-1} = (A - i sum B_mu gamma_mu) / (A^2 + |B|^2)
    Minv = A[..., None, None] * np.eye(4)
    for mu in range(4):
        Minv = Minv - 1j * B[mu][..., None, None] * g[mu]
    Minv = Minv / den[..., None, None]
    xt = np.einsum("...ab,...bc->...ac", Minv, bt)
    x = np.fft.ifftn(xt, axes=(0, 1, 2, 3)) / tw
    return x.reshape(-1, 4, 3)
