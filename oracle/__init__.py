"""FP64 CPU oracle for the Wilson fermion matrix D = 1 - kappa*H, the clover matrix
D_clov = D + F, and their solvers.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the CPU
baseline leg of bench.py.  The product library never imports, links or calls it,
and it shares no code with the GPU path.

The arithmetic lives in oracle.c (Eq. (1) of Sec. 2.1 written out with dense 4x4
gamma matrices on the full lattice; the clover term of Sec. 2.1.2 as a dense 12x12
site matrix).  This module adds ctypes marshalling and a
few numpy helpers that are definitions rather than algorithms: the parity mask,
the dense matrix assembled column by column, and the FP16 per-site-scale codec.

Arrays are numpy complex128 in the canonical layout: spinors (V, 4, 3) with
site s = x + Lx*(y + Ly*(z + Lz*t)), links (V, 4, 3, 3) with mu = 0..3 <-> x,y,z,t.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    sig = {
        "oracle_gamma": (None, [ctypes.c_int, _dp]),
        "oracle_hop": (None, [_dp, _dp, _dp, _i32p]),
        "oracle_apply_D": (None, [_dp, _dp, _dp, ctypes.c_double, _i32p]),
        "oracle_dslash": (None, [_dp, _dp, _dp, ctypes.c_double, _i32p, ctypes.c_int32]),
        "oracle_hop_sites": (None, [_dp, _dp, _dp, _i32p, _i64p, ctypes.c_int64]),
        "oracle_gamma5": (None, [_dp, _dp, ctypes.c_int64]),
        "oracle_eo_prepare": (None, [_dp, _dp, _dp, ctypes.c_double, _i32p]),
        "oracle_eo_reconstruct": (None, [_dp, _dp, _dp, ctypes.c_double, _i32p]),
        "oracle_apply_Mee": (None, [_dp, _dp, _dp, ctypes.c_double, _i32p, ctypes.c_int32]),
        "oracle_solve": (ctypes.c_int, [_dp, _dp, _dp, ctypes.c_double, _i32p, ctypes.c_double,
                                        ctypes.c_int32, ctypes.c_int32, _dp]),
        "oracle_triad": (ctypes.c_double, [ctypes.c_int64, ctypes.c_int32]),
        "oracle_num_threads": (ctypes.c_int, []),
        "oracle_set_threads": (None, [ctypes.c_int32]),
        "oracle_clover_inverse": (ctypes.c_int, [_dp, _dp, ctypes.c_int64]),
        "oracle_apply_Dclov": (None, [_dp, _dp, _dp, _dp, ctypes.c_double, _i32p]),
        "oracle_clov_eo_prepare": (None, [_dp, _dp, _dp, _dp, ctypes.c_double, _i32p]),
        "oracle_clov_eo_reconstruct": (None, [_dp, _dp, _dp, _dp, ctypes.c_double, _i32p]),
        "oracle_apply_Mee_clov": (None, [_dp, _dp, _dp, _dp, ctypes.c_double, _i32p, ctypes.c_int32]),
        "oracle_solve_clov": (ctypes.c_int, [_dp, _dp, _dp, _dp, ctypes.c_double, _i32p, ctypes.c_double,
                                             ctypes.c_int32, ctypes.c_int32, _dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _dims(dims):
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
    assert d.shape == (4,) and np.all(d >= 2) and np.all(d % 2 == 0), "extents must be even and >= 2"
    return d


def _spinor(a, V):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    assert a.size == 12 * V, a.shape
    return a


def _links(U, V):
    U = np.ascontiguousarray(U, dtype=np.complex128)
    assert U.size == 36 * V, U.shape
    return U


def volume(dims):
    return int(np.prod(dims))


def gamma(idx):
    """Dirac-basis gamma matrix used by the oracle (0..3 = gamma_1..4, 4 = gamma_5)."""
    out = np.zeros((4, 4), np.complex128)
    _load().oracle_gamma(idx, _ptr(out))
    return out


def parity_of_sites(dims):
    """(x+y+z+t) mod 2 for every site in canonical order."""
    Lx, Ly, Lz, Lt = dims
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    return ((x + y + z + t) & 1).reshape(-1)


def hop(psi, U, dims):
    """(H psi) on every site: the bracketed sum of Eq. (1)."""
    d = _dims(dims); V = volume(d)
    psi = _spinor(psi, V); U = _links(U, V)
    out = np.empty((V, 4, 3), np.complex128)
    _load().oracle_hop(_ptr(out), _ptr(psi), _ptr(U), d.ctypes.data_as(_i32p))
    return out


def apply_D(psi, U, kappa, dims):
    """D psi = psi - kappa H psi (Eq. (1))."""
    d = _dims(dims); V = volume(d)
    psi = _spinor(psi, V); U = _links(U, V)
    out = np.empty((V, 4, 3), np.complex128)
    _load().oracle_apply_D(_ptr(out), _ptr(psi), _ptr(U), float(kappa), d.ctypes.data_as(_i32p))
    return out


def dslash(psi, U, kappa, dims, parity, out=None):
    """Entry-point semantics: parity 0/1 -> -kappa*H on parity-p sites (others untouched); 2 -> D psi."""
    d = _dims(dims); V = volume(d)
    psi = _spinor(psi, V); U = _links(U, V)
    out = np.zeros((V, 4, 3), np.complex128) if out is None else np.ascontiguousarray(out, np.complex128).copy()
    _load().oracle_dslash(_ptr(out), _ptr(psi), _ptr(U), float(kappa), d.ctypes.data_as(_i32p), int(parity))
    return out


def hop_sites(psi, U, dims, sites):
    """(H psi)(s) at the listed sites only; returns (n, 4, 3)."""
    d = _dims(dims); V = volume(d)
    psi = _spinor(psi, V); U = _links(U, V)
    sites = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
    out = np.empty((sites.size, 4, 3), np.complex128)
    _load().oracle_hop_sites(_ptr(out), _ptr(psi), _ptr(U), d.ctypes.data_as(_i32p),
                             sites.ctypes.data_as(_i64p), sites.size)
    return out


def gamma5(psi):
    psi = np.ascontiguousarray(psi, np.complex128)
    V = psi.size // 12
    out = np.empty((V, 4, 3), np.complex128)
    _load().oracle_gamma5(_ptr(out), _ptr(psi), V)
    return out


def eo_prepare(b, U, kappa, dims):
    """b'_e = b_e + kappa H_eo b_o on even sites, zero on odd sites."""
    d = _dims(dims); V = volume(d)
    b = _spinor(b, V); U = _links(U, V)
    out = np.empty((V, 4, 3), np.complex128)
    _load().oracle_eo_prepare(_ptr(out), _ptr(b), _ptr(U), float(kappa), d.ctypes.data_as(_i32p))
    return out


def eo_reconstruct(x_even, b, U, kappa, dims):
    """Returns x with x_e from x_even and x_o = b_o + kappa H_oe x_e."""
    d = _dims(dims); V = volume(d)
    x = _spinor(x_even, V).copy(); b = _spinor(b, V); U = _links(U, V)
    _load().oracle_eo_reconstruct(_ptr(x), _ptr(b), _ptr(U), float(kappa), d.ctypes.data_as(_i32p))
    return x.reshape(V, 4, 3)


def apply_Mee(psi, U, kappa, dims, dagger=False):
    """M_ee psi_e = psi_e - kappa^2 H_eo H_oe psi_e (or its adjoint); odd sites of the result are 0."""
    d = _dims(dims); V = volume(d)
    psi = _spinor(psi, V); U = _links(U, V)
    out = np.empty((V, 4, 3), np.complex128)
    _load().oracle_apply_Mee(_ptr(out), _ptr(psi), _ptr(U), float(kappa), d.ctypes.data_as(_i32p), int(dagger))
    return out


METHODS = {"bicgstab_full": 0, "bicgstab_eo": 1, "cgls_eo": 2}


def solve(b, U, kappa, dims, tol, maxiter, method="bicgstab_eo", x0=None):
    """Solve D x = b; returns (x, status, true_rel_residual).

    status >= 0 is the iteration count, -1 not converged, -2 breakdown.
    """
    d = _dims(dims); V = volume(d)
    b = _spinor(b, V); U = _links(U, V)
    x = np.zeros((V, 4, 3), np.complex128) if x0 is None else _spinor(x0, V).copy().reshape(V, 4, 3)
    tr = ctypes.c_double(0.0)
    st = _load().oracle_solve(_ptr(x), _ptr(b), _ptr(U), float(kappa), d.ctypes.data_as(_i32p), float(tol),
                              int(maxiter), METHODS[method], ctypes.byref(tr))
    return x, int(st), float(tr.value)


# ---- clover fermion matrix (Sec. 2.1.2): D_clov = D_W + F(x) delta_{x,y} ----
# F is an input array (V, 12, 12) complex128, Hermitian per site, rows and columns
# 3*spin + colour in the Dirac basis.

def _clover(F, V):
    F = np.ascontiguousarray(F, dtype=np.complex128)
    assert F.size == 144 * V, F.shape
    return F


def clover_inverse(F):
    """(1 + F(x))^-1 per site, (V, 12, 12); raises if a site matrix is singular."""
    F = np.ascontiguousarray(F, dtype=np.complex128)
    V = F.size // 144
    out = np.empty((V, 12, 12), np.complex128)
    if _load().oracle_clover_inverse(_ptr(out), _ptr(F), V) != 0:
        raise ValueError("singular 1 + F")
    return out


def apply_Dclov(psi, U, F, kappa, dims):
    """D_clov psi = (1 + F) psi - kappa H psi."""
    d = _dims(dims); V = volume(d)
    psi = _spinor(psi, V); U = _links(U, V); F = _clover(F, V)
    out = np.empty((V, 4, 3), np.complex128)
    _load().oracle_apply_Dclov(_ptr(out), _ptr(psi), _ptr(U), _ptr(F), float(kappa), d.ctypes.data_as(_i32p))
    return out


def clov_eo_prepare(b, U, F, kappa, dims):
    """b'_e = b_e + kappa H_eo T_oo^-1 b_o on even sites (odd sites 0)."""
    d = _dims(dims); V = volume(d)
    b = _spinor(b, V); U = _links(U, V); F = _clover(F, V)
    out = np.empty((V, 4, 3), np.complex128)
    _load().oracle_clov_eo_prepare(_ptr(out), _ptr(b), _ptr(U), _ptr(F), float(kappa), d.ctypes.data_as(_i32p))
    return out


def clov_eo_reconstruct(x_even, b, U, F, kappa, dims):
    """x with x_o = T_oo^-1 (b_o + kappa H_oe x_e) written on the odd sites."""
    d = _dims(dims); V = volume(d)
    x = _spinor(x_even, V).copy(); b = _spinor(b, V); U = _links(U, V); F = _clover(F, V)
    _load().oracle_clov_eo_reconstruct(_ptr(x), _ptr(b), _ptr(U), _ptr(F), float(kappa), d.ctypes.data_as(_i32p))
    return x.reshape(V, 4, 3)


def apply_Mee_clov(psi, U, F, kappa, dims, dagger=False):
    """M_ee psi_e = T_ee psi_e - kappa^2 H_eo T_oo^-1 H_oe psi_e (odd sites of psi ignored)."""
    d = _dims(dims); V = volume(d)
    psi = _spinor(psi, V); U = _links(U, V); F = _clover(F, V)
    out = np.empty((V, 4, 3), np.complex128)
    _load().oracle_apply_Mee_clov(_ptr(out), _ptr(psi), _ptr(U), _ptr(F), float(kappa), d.ctypes.data_as(_i32p),
                                  int(bool(dagger)))
    return out


def solve_clov(b, U, F, kappa, dims, tol, maxiter, method="bicgstab_eo"):
    """Solve D_clov x = b; returns (x, status, true_rel_residual) as solve()."""
    d = _dims(dims); V = volume(d)
    b = _spinor(b, V); U = _links(U, V); F = _clover(F, V)
    x = np.zeros((V, 4, 3), np.complex128)
    tr = ctypes.c_double(0.0)
    st = _load().oracle_solve_clov(_ptr(x), _ptr(b), _ptr(U), _ptr(F), float(kappa), d.ctypes.data_as(_i32p),
                                   float(tol), int(maxiter), METHODS[method], ctypes.byref(tr))
    return x, int(st), float(tr.value)


def dense_D(U, kappa, dims):
    """The full matrix D (12V x 12V) assembled column by column from apply_D (tiny lattices only)."""
    d = _dims(dims); V = volume(d)
    n = 12 * V
    assert n <= 4096, "dense assembly is for tiny lattices"
    M = np.empty((n, n), np.complex128)
    e = np.zeros(n, np.complex128)
    for j in range(n):
        e[:] = 0
        e[j] = 1
        M[:, j] = apply_D(e, U, kappa, d).reshape(-1)
    return M


def fp16_encode(psi):
    """Per-site FP16 codec (definition): values rounded to FP32, s = max |component| over
    the 24 reals of the site (FP32), h = fp16_rne(fp32(v / s)); s = 0 encodes zeros.
    Returns (h: float16 (V, 24), s: float32 (V,))."""
    a = np.ascontiguousarray(psi, np.complex128).reshape(-1, 12)
    re = np.stack([a.real, a.imag], axis=-1).reshape(-1, 24).astype(np.float32)
    s = np.max(np.abs(re), axis=1).astype(np.float32)
    safe = np.where(s > 0, s, np.float32(1.0)).astype(np.float32)
    q = (re / safe[:, None]).astype(np.float32)
    q = np.where(s[:, None] > 0, q, np.float32(0.0))
    return q.astype(np.float16), s


def fp16_decode(h, s):
    """Inverse of fp16_encode: value = fp32(h) * s, as complex128 (V, 4, 3)."""
    v = h.astype(np.float32) * s[:, None].astype(np.float32)
    v = v.astype(np.float64).reshape(-1, 12, 2)
    return (v[..., 0] + 1j * v[..., 1]).reshape(-1, 4, 3)


def triad_gbps(n=1 << 26, reps=10):
    """Host triad bandwidth (GB/s) with the oracle's OpenMP threads."""
    secs = _load().oracle_triad(int(n), int(reps))
    return 3 * 8 * n * reps / secs / 1e9


def num_threads():
    return int(_load().oracle_num_threads())


def set_threads(n):
    """OpenMP threads for later oracle calls (timing only)."""
    _load().oracle_set_threads(int(n))


# block BiCGStab for several right-hand sides of one matrix (kept in its own module)
from .block_krylov import BlockBreakdown, block_bicgstab, solve_block  # noqa: E402,F401
