"""Host-side checks on the CPU (no GPU).

1. The site indexing of the kernels (checkerboard decode, the eight neighbour indices of
   the hop, the plane-blocked visiting orders and the XCD-contiguous block order; the
   library's own functions, compiled for the host) replayed by wilson_index_check on every
   lattice shape the tests and the benchmark use: all in range, at the coordinates the
   lattice's definition gives, and permutations where they should be.
2. The host code of the library (runtime, solver, C ABI, index check) rebuilt with
   AddressSanitizer and UndefinedBehaviorSanitizer and driven through its host paths
   (argument validation, footprints, the index check, error reporting, a context on a
   machine without a GPU) in a subprocess that has the sanitizer runtime preloaded; any
   report fails the test."""
import glob
import os
import re
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def lattice_shapes():
    """Every 4-tuple of even extents >= 2 written in the tests or the benchmark."""
    shapes = set()
    files = glob.glob(os.path.join(ROOT, "tests", "*.py")) + [os.path.join(ROOT, "bench.py")]
    for f in files:
        for m in re.finditer(r"\(\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+)\s*\)", open(f).read()):
            d = tuple(int(v) for v in m.groups())
            if all(v >= 2 and v % 2 == 0 for v in d):
                shapes.add(d)
    return sorted(shapes, key=lambda d: d[0] * d[1] * d[2] * d[3])


def test_shape_scan_finds_the_benchmark_lattices():
    s = lattice_shapes()
    for d in [(2, 2, 2, 2), (4, 4, 4, 8), (8, 8, 8, 8), (16, 16, 16, 32), (24, 24, 24, 48), (32, 32, 32, 64),
              (48, 48, 48, 96), (6, 4, 2, 10)]:
        assert d in s


@pytest.mark.parametrize("dims", lattice_shapes(), ids=lambda d: "x".join(map(str, d)))
def test_kernel_index_maps(dims):
    from paper_1811_00893_amd import _lib
    st = _lib.wilson_index_check(dims)
    assert st == 0, _lib.wilson_last_error()


def test_index_check_rejects_invalid_lattices():
    from paper_1811_00893_amd import _lib
    assert _lib.wilson_index_check((4, 3, 4, 4)) == _lib.WILSON_INVALID_ARG
    assert _lib.wilson_index_check(None) == _lib.WILSON_INVALID_ARG


SAN_DRIVER = textwrap.dedent(r'''
    import ctypes, sys
    lib = ctypes.CDLL(sys.argv[1])
    I4 = ctypes.c_int32 * 4
    lib.wilson_last_error.restype = ctypes.c_char_p
    lib.wilson_strerror.restype = ctypes.c_char_p
    lib.wilson_version.restype = ctypes.c_char_p
    lib.wilson_footprint_bytes.restype = ctypes.c_size_t
    lib.wilson_footprint_bytes.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
    lib.wilson_gauge_footprint_bytes.restype = ctypes.c_size_t
    lib.wilson_gauge_footprint_bytes.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int32]
    INVALID = -1
    print(lib.wilson_version().decode())
    for code in range(-8, 2):
        assert lib.wilson_strerror(code)
    # the index replay, on shapes small enough for the instrumented build
    for d in [(2, 2, 2, 2), (2, 4, 2, 6), (4, 4, 4, 4), (4, 4, 4, 8), (6, 4, 2, 10), (4, 6, 8, 10), (8, 8, 8, 8)]:
        assert lib.wilson_index_check(I4(*d)) == 0, (d, lib.wilson_last_error())
    assert lib.wilson_index_check(I4(4, 4, 4, 5)) == INVALID
    assert lib.wilson_index_check(None) == INVALID
    # footprints for every precision and solver, nrhs over its range, and invalid input
    class Opts(ctypes.Structure):
        pass
    nbytes = set()
    for d in [(4, 4, 4, 8), (16, 16, 16, 32), (48, 48, 48, 96)]:
        for nrhs in (1, 2, 12, 64):
            nbytes.add(lib.wilson_footprint_bytes(I4(*d), nrhs, None))
        for prec in (1, 2, 3, 4, 7):
            assert lib.wilson_gauge_footprint_bytes(I4(*d), prec, 12) > 0
            assert lib.wilson_gauge_footprint_bytes(I4(*d), prec, 18) > 0
    assert 0 not in nbytes
    assert lib.wilson_footprint_bytes(I4(4, 4, 4, 8), 0, None) == 0
    assert lib.wilson_footprint_bytes(I4(4, 4, 4, 8), 65, None) == 0
    assert lib.wilson_footprint_bytes(I4(3, 4, 4, 8), 1, None) == 0
    assert lib.wilson_footprint_bytes(None, 1, None) == 0
    assert lib.wilson_gauge_footprint_bytes(I4(4, 4, 4, 8), 1, 10) == 0
    # the plain entry points reject bad arguments before any device work
    buf = (ctypes.c_double * (24 * 4 * 4 * 4 * 8))()
    U = (ctypes.c_double * (72 * 4 * 4 * 4 * 8))()
    lib.wilson_dslash.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                  ctypes.c_void_p, ctypes.c_int32]
    lib.wilson_solve.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                 ctypes.c_void_p, ctypes.c_double, ctypes.c_int32]
    assert lib.wilson_dslash(None, buf, U, 0.1, I4(4, 4, 4, 8), 2) == INVALID
    assert lib.wilson_dslash(buf, buf, U, 0.1, I4(4, 4, 4, 7), 2) == INVALID
    assert lib.wilson_solve(buf, buf, None, 0.1, I4(4, 4, 4, 8), 1e-10, 100) == INVALID
    assert lib.wilson_solve(buf, buf, U, 0.1, I4(4, 4, 4, 8), -1.0, 100) == INVALID
    assert lib.wilson_last_error()
    # calls on a NULL context or field
    lib.wilson_solve_ex.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int32] + [ctypes.c_void_p] * 4
    assert lib.wilson_solve_ex(None, None, buf, buf, 1, None, None, None, None) == INVALID
    # a context: created where a GPU is visible, a clean error where none is
    ctx = ctypes.c_void_p()
    st = lib.wilson_context_create(ctypes.byref(ctx), None)
    if st == 0:
        assert lib.wilson_context_destroy(ctx) == 0
    else:
        assert st < 0 and lib.wilson_last_error()
    print("sanitized host paths ok", flush=True)
''')


def test_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    from paper_1811_00893_amd.csrc import build
    runtime = build.sanitizer_runtime()
    assert runtime, "the compiler's AddressSanitizer runtime was not found"
    lib = build.build_sanitized()
    script = tmp_path / "drive.py"
    script.write_text(SAN_DRIVER)
    env = dict(os.environ, LD_PRELOAD=runtime, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, str(script), lib], env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "sanitized host paths ok" in r.stdout


def test_vector_and_block_kernels_do_not_spill():
    """The solver's vector kernels (fused BLAS-1 updates, reductions, finalize) and the block
    BiCGStab kernels hold one element per thread and an s x s matrix in LDS: none of them
    needs scratch.  A spill there (the coefficient matrix once went into registers, 256 VGPRs
    and 868 bytes of scratch per lane, when the field pointers changed address space) slows
    them 2-4x with no change in results, so only the compiler's resource report shows it."""
    sys.path.insert(0, os.path.join(ROOT, "paper_1811_00893_amd", "csrc"))
    import build
    allowed = {"_ZN2wl17block_gram_kernelILi16EEEvNS_9BlockArgsE"}  # 4x4 tiles of a 16-column block
    for src in ("blas.hip", "block.hip"):
        usage = build.resource_usage(src)
        assert len(usage) >= 5, (src, usage)
        spills = {k: v for k, v in usage.items() if v.get("scratch", 0) > 0 and k not in allowed}
        assert not spills, (src, spills)
