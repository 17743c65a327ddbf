"""Host-side checks of the C ABI that need no GPU: every declared symbol is exported,
status strings, and argument validation that fails before any device work."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ntt_mi355x.h")
LIB = os.environ.get("NTT_MI355X_LIB") or os.path.join(ROOT, "paper_2012_01968_amd", "libntt_mi355x.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ntt_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("library not built: run python paper_2012_01968_amd/build.py")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ntt_plan_create", "ntt_plan_destroy", "ntt_plan_get_roots", "ntt_forward", "ntt_inverse",
                     "ntt_pointwise_mul", "ntt_polymul_negacyclic", "ntt_status_string"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in declared_functions():
        assert name in exported, name
        assert getattr(lib, name) is not None


def test_status_strings(lib):
    lib.ntt_status_string.restype = ctypes.c_char_p
    want = {0: b"NTT_OK", -1: b"NTT_ERR_ARG", -2: b"NTT_ERR_N", -3: b"NTT_ERR_PRIME", -4: b"NTT_ERR_NOMEM",
            -5: b"NTT_ERR_HIP", -6: b"NTT_ERR_UNSUPPORTED"}
    for code, name in want.items():
        assert lib.ntt_status_string(code) == name


class _Opts(ctypes.Structure):
    _fields_ = [("twiddle_mode", ctypes.c_int32), ("ot_stages", ctypes.c_int32),
                ("ot_log2_base", ctypes.c_int32), ("log2_n1", ctypes.c_int32),
                ("kernel_path", ctypes.c_int32), ("use_autotune", ctypes.c_int32),
                ("tune_polys", ctypes.c_int32), ("order", ctypes.c_int32), ("log2_radix", ctypes.c_int32),
                ("word_bits", ctypes.c_int32), ("r1", ctypes.c_int32), ("wg_size", ctypes.c_int32),
                ("col_width", ctypes.c_int32), ("reserved", ctypes.c_int32)]


def _create(lib, N, primes, opts=None):
    lib.ntt_plan_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint32,
                                    ctypes.POINTER(ctypes.c_uint64), ctypes.c_uint32, ctypes.POINTER(_Opts)]
    lib.ntt_plan_create.restype = ctypes.c_int
    h = ctypes.c_void_p(1234)
    arr = (ctypes.c_uint64 * max(1, len(primes)))(*primes)
    rc = lib.ntt_plan_create(ctypes.byref(h), N, arr, len(primes), ctypes.byref(opts) if opts else None)
    return rc, h.value


def test_argument_errors_are_synchronous(lib):
    import synth
    q = synth.gen_primes(5, 1 << 17, 60, 1)[0]   # 60-bit prime, 1 mod 2^18
    assert _create(lib, 0, [q]) == (-2, None)
    assert _create(lib, 3, [q]) == (-2, None)
    assert _create(lib, 1 << 18, [q]) == (-2, None)
    assert _create(lib, 1 << 10, [q + 2]) == (-3, None)           # not 1 mod 2N
    assert _create(lib, 1 << 10, [q, q]) == (-3, None)             # repeated
    assert _create(lib, 1 << 10, [(1 << 62) + 1]) == (-3, None)    # too large
    assert _create(lib, 1 << 10, [1 + (1 << 11) * 3 * 5]) == (-3, None)  # 30721 = 31*991: composite, 1 mod 2N
    assert _create(lib, 1 << 10, []) == (-1, None)
    o = _Opts()
    o.reserved = 1
    assert _create(lib, 1 << 10, [q], o) == (-1, None)
    o = _Opts(0, 0, 0, 0, 0, 0, 0, 0, 0, 16)
    assert _create(lib, 1 << 10, [q], o) == (-1, None)             # word_bits is 0, 32 or 64
    o = _Opts(0, 0, 0, 0, 0, 0, 0, 0, 0, 32)
    assert _create(lib, 1 << 10, [q], o) == (-3, None)             # 32-bit words need q < 2^30
    o = _Opts(2, 2, 10, 0, 0, 0, 0, 0, 0, 32)
    assert _create(lib, 1 << 16, [(1 << 29) + 1], o) == (-6, None) # 32-bit plans take table twiddles
    o = _Opts(0, 0, 0, 0, 0, 0, 0, 2)
    assert _create(lib, 1 << 10, [q], o) == (-1, None)             # order is BITREV or NATURAL
    o = _Opts(0, 0, 0, 0, 0, 2)
    assert _create(lib, 1 << 10, [q], o) == (-1, None)             # use_autotune is 0 or 1
    o = _Opts(0, 0, 0, 0, 0, 1, -1)
    assert _create(lib, 1 << 10, [q], o) == (-1, None)             # negative tune_polys
    o = _Opts(2, 2, 10, 0)
    assert _create(lib, 1 << 10, [q], o) == (-6, None)             # OT base must be below N
    o = _Opts(0, 0, 0, 11)
    assert _create(lib, 1 << 16, [q], o) == (-6, None)             # no column pass of 2^11
    o = _Opts(0, 0, 0, 0, 5)
    assert _create(lib, 1 << 16, [q], o) == (-1, None)             # kernel_path out of range
    o = _Opts(0, 0, 0, 0, 4, 0, 0, 0, 1)
    assert _create(lib, 1 << 16, [q], o) == (-1, None)             # register path: radix 2^2 .. 2^5
    o = _Opts(0, 0, 0, 0, 1, 0, 0, 0, 3)
    assert _create(lib, 1 << 16, [q], o) == (-1, None)             # log2_radix only with the register path
    o = _Opts(2, 2, 10, 0, 3)
    assert _create(lib, 1 << 16, [q], o) == (-6, None)             # radix-2 path: table twiddles only
    o = _Opts(0, 0, 0, 9, 2)
    assert _create(lib, 1 << 16, [q], o) == (-6, None)             # no fused 2^9 x 2^7 shape
    o = _Opts(0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 2)
    assert _create(lib, 1 << 16, [q], o) == (-1, None)             # r1 is 4 or 8
    o = _Opts(0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 96)
    assert _create(lib, 1 << 16, [q], o) == (-1, None)             # wg_size is 64, 128 or 256
    o = _Opts(0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 512)
    assert _create(lib, 1 << 16, [q], o) == (-1, None)             # col_width is 16 .. 256
    o = _Opts(0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 16)
    assert _create(lib, 1 << 10, [q], o) == (-6, None)             # one-pass plan: no column tile
    o = _Opts(0, 0, 0, 0, 3, 0, 0, 0, 0, 0, 4)
    assert _create(lib, 1 << 16, [q], o) == (-6, None)             # tiles belong to the split path
    o = _Opts(0, 0, 0, 0, 0, 0, 0, 0, 0, 32, 4)
    assert _create(lib, 1 << 16, [(1 << 29) + 1], o) == (-6, None) # and to 64-bit plans
    lib.ntt_forward.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p]
    lib.ntt_forward.restype = ctypes.c_int
    assert lib.ntt_forward(None, None, 1, None) == -1


def test_device_copy_argument_errors(lib):
    vp = ctypes.c_void_p
    lib.ntt_device_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
    lib.ntt_device_copy.restype = ctypes.c_int
    assert lib.ntt_device_copy(None, None, 0, None) == 0              # nothing to copy
    assert lib.ntt_device_copy(None, 4096, 64, None) == -1            # null destination
    assert lib.ntt_device_copy(8192, None, 64, None) == -1            # null source
    assert lib.ntt_device_copy(8200, 4096, 64, None) == -1            # misaligned
    assert lib.ntt_device_copy(8192, 4096, 40, None) == -1            # not a multiple of 16
    assert lib.ntt_device_copy(8192, 4096, 1 << 35, None) == -1       # too large
    assert lib.ntt_device_copy(4096 + 32, 4096, 64, None) == -1       # overlapping


def test_batch_argument_errors(lib):
    vp = ctypes.c_void_p
    lib.ntt_batch_create.argtypes = [ctypes.POINTER(vp), vp, ctypes.c_uint32]
    lib.ntt_batch_assign.argtypes = [vp, vp, ctypes.c_uint32, vp]
    lib.ntt_batch_run.argtypes = [vp, ctypes.c_int32, vp]
    lib.ntt_batch_destroy.argtypes = [vp]
    h = vp(99)
    assert lib.ntt_batch_create(None, None, 0) == -1
    assert lib.ntt_batch_create(ctypes.byref(h), None, 0) == -1 and h.value is None
    assert lib.ntt_batch_assign(None, None, 0, None) == -1
    assert lib.ntt_batch_run(None, 0, None) == -1
    assert lib.ntt_batch_destroy(None) == 0


@pytest.mark.parametrize("order", ["package first", "torch first"])
def test_one_hip_runtime_whatever_the_import_order(order):
    """The binding and PyTorch must share one HIP runtime: a second libamdhip64 in the
    process cannot use device pointers or streams of the first (plan creation then fails
    with hipGetDevice errors)."""
    import sys
    pytest.importorskip("torch")
    imports = "import paper_2012_01968_amd, torch" if order == "package first" else \
        "import torch, paper_2012_01968_amd"
    code = imports + "; print(len({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))"
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip() == "1"
