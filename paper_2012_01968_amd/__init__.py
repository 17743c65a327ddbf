"""Batched negacyclic NTT for MI355X (gfx950): Python binding of libntt_mi355x.so.

Every function here marshals arguments for the C entry point of the same name
(include/ntt_mi355x.h); all arithmetic runs in the HIP kernels.  Device buffers may be
given as torch tensors (int64 or uint64, on the GPU; their storage is read as uint64)
or as raw integer device addresses.  Streams may be torch streams, raw hipStream_t
integers, or None for torch's current stream.

Loading fails loudly (ImportError) when the built library is missing: there is no
fallback path.  Build it with ``python paper_2012_01968_amd/build.py``.
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "NttError", "Plan", "ntt_plan_create", "ntt_plan_destroy", "ntt_plan_get_roots", "ntt_plan_get_info",
    "ntt_forward", "ntt_inverse", "ntt_forward_pass", "ntt_inverse_pass", "ntt_plan_num_passes", "ntt_plan_tuned",
    "ntt_plan_order", "ORDER_BITREV", "ORDER_NATURAL",
    "ntt_pointwise_mul", "ntt_polymul_negacyclic", "ntt_status_string",
    "Batch", "ntt_batch_create", "ntt_batch_run", "ntt_batch_destroy", "ntt_batch_assign", "OP_FORWARD", "OP_INVERSE",
    "OP_FORWARD_INVERSE", "OP_MULKEY", "BATCH_PLAIN", "BATCH_GROUPED", "BATCH_GRAPH", "BATCH_GRAPH_BRANCHED",
    "library_path", "TWIDDLE_AUTO", "TWIDDLE_TABLE", "TWIDDLE_OT", "PATH_AUTO", "PATH_SPLIT", "PATH_FUSED",
    "PATH_RADIX2", "PATH_REGISTER", "ntt_plan_log2_radix", "ntt_forward_u32", "ntt_inverse_u32",
    "ntt_pointwise_mul_u32", "ntt_polymul_negacyclic_u32", "ntt_plan_word_bits", "ntt_crt_words",
    "ntt_rns_decompose", "ntt_crt_reconstruct", "ntt_polymul_negacyclic_noalloc", "ntt_polymul_noalloc_max_words",
    "ntt_device_copy",
]

TWIDDLE_AUTO, TWIDDLE_TABLE, TWIDDLE_OT = 0, 1, 2
PATH_AUTO, PATH_SPLIT, PATH_FUSED, PATH_RADIX2, PATH_REGISTER = 0, 1, 2, 3, 4
OP_FORWARD, OP_INVERSE, OP_FORWARD_INVERSE, OP_MULKEY = 1, 2, 3, 4
BATCH_PLAIN, BATCH_GROUPED, BATCH_GRAPH, BATCH_GRAPH_BRANCHED = 0, 1, 2, 3
ORDER_BITREV, ORDER_NATURAL = 0, 1

_HERE = os.path.dirname(os.path.abspath(__file__))
# NTT_MI355X_LIB selects another build of the library (e.g. a tuning variant).
_LIB_PATH = os.environ.get("NTT_MI355X_LIB") or os.path.join(_HERE, "libntt_mi355x.so")


def library_path() -> str:
    return _LIB_PATH


if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is not built; run `python paper_2012_01968_amd/build.py`")


def _share_torch_hip_runtime() -> None:
    """Load PyTorch's own HIP runtime first, if PyTorch is installed, so that the library
    binds to the same runtime as the tensors and streams it is handed.  PyTorch-ROCm ships
    its own libamdhip64; if the library were loaded first it would bring in the system
    copy, and a process with two HIP runtimes cannot pass device pointers between them."""
    import importlib.util
    try:
        spec = importlib.util.find_spec("torch")
    except (ImportError, ValueError):
        return
    if spec is None or not spec.submodule_search_locations:
        return
    for root in spec.submodule_search_locations:
        path = os.path.join(root, "lib", "libamdhip64.so")
        if os.path.exists(path):
            ctypes.CDLL(path, mode=ctypes.RTLD_GLOBAL)
            return


_share_torch_hip_runtime()
_lib = ctypes.CDLL(_LIB_PATH)


class _Opts(ctypes.Structure):
    _fields_ = [("twiddle_mode", ctypes.c_int32), ("ot_stages", ctypes.c_int32),
                ("ot_log2_base", ctypes.c_int32), ("log2_n1", ctypes.c_int32),
                ("kernel_path", ctypes.c_int32), ("use_autotune", ctypes.c_int32),
                ("tune_polys", ctypes.c_int32), ("order", ctypes.c_int32), ("log2_radix", ctypes.c_int32),
                ("word_bits", ctypes.c_int32), ("r1", ctypes.c_int32), ("wg_size", ctypes.c_int32),
                ("col_width", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_vp = ctypes.c_void_p
_u32 = ctypes.c_uint32


class _Job(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("d_data", ctypes.c_void_p), ("n_polys", ctypes.c_uint32),
                ("n_limbs", ctypes.c_uint32), ("op", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("d_key", ctypes.c_void_p)]


_u64p = ctypes.POINTER(ctypes.c_uint64)
_lib.ntt_plan_create.argtypes = [ctypes.POINTER(_vp), _u32, _u64p, _u32, ctypes.POINTER(_Opts)]
_lib.ntt_plan_destroy.argtypes = [_vp]
_lib.ntt_plan_get_roots.argtypes = [_vp, _u64p]
_lib.ntt_plan_get_info.argtypes = [_vp, ctypes.POINTER(_u32), ctypes.POINTER(_u32), ctypes.POINTER(_u32),
                                   ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int32)]
_lib.ntt_plan_get_tiles.argtypes = [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32)]
_lib.ntt_forward.argtypes = [_vp, _vp, _u32, _vp]
_lib.ntt_inverse.argtypes = [_vp, _vp, _u32, _vp]
_lib.ntt_forward_pass.argtypes = [_vp, _vp, _u32, _u32, _vp]
_lib.ntt_inverse_pass.argtypes = [_vp, _vp, _u32, _u32, _vp]
_lib.ntt_plan_num_passes.argtypes = [_vp]
_lib.ntt_plan_num_passes.restype = _u32
_lib.ntt_plan_tuned.argtypes = [_vp]
_lib.ntt_plan_order.argtypes = [_vp]
_lib.ntt_plan_order.restype = ctypes.c_int32
_lib.ntt_plan_log2_radix.argtypes = [_vp]
_lib.ntt_plan_log2_radix.restype = ctypes.c_int32
_lib.ntt_plan_tuned.restype = ctypes.c_int32
_lib.ntt_pointwise_mul.argtypes = [_vp, _vp, _vp, _vp, _u32, _vp]
_lib.ntt_polymul_negacyclic.argtypes = [_vp, _vp, _vp, _vp, _u32, _vp]
_lib.ntt_polymul_negacyclic_noalloc.argtypes = [_vp, _vp, _vp, _vp, _u32, _vp]
_lib.ntt_polymul_noalloc_max_words.argtypes = []
_lib.ntt_polymul_noalloc_max_words.restype = ctypes.c_uint64
for _f in ("ntt_forward_u32", "ntt_inverse_u32"):
    getattr(_lib, _f).argtypes = [_vp, _vp, _u32, _vp]
    getattr(_lib, _f).restype = ctypes.c_int
for _f in ("ntt_pointwise_mul_u32", "ntt_polymul_negacyclic_u32"):
    getattr(_lib, _f).argtypes = [_vp, _vp, _vp, _vp, _u32, _vp]
    getattr(_lib, _f).restype = ctypes.c_int
_lib.ntt_plan_word_bits.argtypes = [_vp]
_lib.ntt_plan_word_bits.restype = ctypes.c_int32
_lib.ntt_crt_words.argtypes = [_vp]
_lib.ntt_crt_words.restype = _u32
_lib.ntt_rns_decompose.argtypes = [_vp, _vp, _u32, _vp, _u32, _vp]
_lib.ntt_rns_decompose.restype = ctypes.c_int
_lib.ntt_crt_reconstruct.argtypes = [_vp, _vp, _vp, _u32, _vp]
_lib.ntt_crt_reconstruct.restype = ctypes.c_int
_lib.ntt_batch_create.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(_Job), _u32]
_lib.ntt_batch_run.argtypes = [_vp, ctypes.c_int32, _vp]
_lib.ntt_batch_assign.argtypes = [_vp, ctypes.POINTER(_Job), _u32, _vp]
_lib.ntt_batch_destroy.argtypes = [_vp]
_lib.ntt_device_copy.argtypes = [_vp, _vp, ctypes.c_size_t, _vp]
_lib.ntt_device_copy.restype = ctypes.c_int
_lib.ntt_status_string.argtypes = [ctypes.c_int]
_lib.ntt_status_string.restype = ctypes.c_char_p
_lib.ntt_last_error.argtypes = []
_lib.ntt_last_error.restype = ctypes.c_char_p
for _f in ("ntt_plan_create", "ntt_plan_destroy", "ntt_plan_get_roots", "ntt_plan_get_info", "ntt_forward",
           "ntt_inverse", "ntt_forward_pass", "ntt_inverse_pass", "ntt_pointwise_mul", "ntt_polymul_negacyclic",
           "ntt_batch_create", "ntt_batch_run", "ntt_batch_destroy", "ntt_batch_assign"):
    getattr(_lib, _f).restype = ctypes.c_int


class NttError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.ntt_last_error().decode(errors="replace")
        super().__init__(f"{where}: {ntt_status_string(status)}: {msg}")


def _check(status: int, where: str) -> None:
    if status != 0:
        raise NttError(status, where)


def ntt_device_copy(dst, src, stream=None) -> None:
    """Copy tensor `src` into `dst` (same byte size, a multiple of 16) with the library's
    one-pass copy kernel: the memory-rate yardstick of the measurements, not part of the
    transform."""
    for t, w in ((dst, "dst"), (src, "src")):
        if not getattr(t, "is_cuda", False) or not t.is_contiguous():
            raise ValueError(f"{w} must be a contiguous tensor in GPU memory")
    nbytes = dst.numel() * dst.element_size()
    if src.numel() * src.element_size() != nbytes:
        raise ValueError("dst and src differ in size")
    _check(_lib.ntt_device_copy(int(dst.data_ptr()), int(src.data_ptr()), nbytes, _stream(stream)),
           "ntt_device_copy")


def ntt_status_string(status: int) -> str:
    return _lib.ntt_status_string(status).decode()


class Plan:
    """Owns an ntt_plan_t; destroyed explicitly or when garbage-collected."""

    def __init__(self, handle: int, N: int, L: int):
        self.handle = handle
        self.N = N
        self.L = L

    def destroy(self) -> None:
        if self.handle:
            _check(_lib.ntt_plan_destroy(self.handle), "ntt_plan_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _addr(buf, need: int | None = None, what: str = "buffer", esize: int = 8) -> int:
    """Device address of `buf` for the C ABI.  A raw integer is passed through as given (the
    caller vouches for it).  A tensor must live on the GPU, hold integers of `esize` bytes, be
    contiguous and have at least `need` elements: anything else would reach the kernels as a
    pointer to memory they cannot address or to too few elements."""
    if buf is None:
        raise ValueError(f"{what} is None")
    if isinstance(buf, int):
        return buf
    if not getattr(buf, "is_cuda", False):
        raise ValueError(f"{what} must be a tensor in GPU memory")
    if buf.element_size() != esize or buf.dtype.is_floating_point or buf.dtype.is_complex:
        raise ValueError(f"{what} must hold {8 * esize}-bit integers, not {buf.dtype}")
    if not buf.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if need is not None and buf.numel() < need:
        raise ValueError(f"{what} holds {buf.numel()} elements; the call needs {need}")
    return int(buf.data_ptr())


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream) or None
    if isinstance(stream, int):
        return stream or None
    return int(stream.cuda_stream) or None


def _polys(plan: Plan, buf, n_polys) -> int:
    if n_polys is not None:
        if int(n_polys) < 1:
            raise ValueError("n_polys must be at least 1")
        return int(n_polys)
    if isinstance(buf, int):
        raise ValueError("n_polys is required when a buffer is given as a raw address")
    numel = buf.numel()
    per = plan.N * plan.L
    if numel == 0 or numel % per:
        raise ValueError(f"buffer of {numel} elements is not a whole number of [L][N] polynomials")
    return numel // per


def _batch_addrs(plan: Plan, bufs, names, n_polys, esize: int = 8):
    """n_polys and the addresses of same-shaped [n_polys][L][N] operands."""
    n = _polys(plan, bufs[0], n_polys)
    need = n * plan.L * plan.N
    return n, [_addr(b, need, w, esize) for b, w in zip(bufs, names)]


def ntt_plan_create(N: int, primes, *, twiddle_mode: int = 0, ot_stages: int = 0, ot_log2_base: int = 0,
                    log2_n1: int = 0, kernel_path: int = 0, use_autotune: int = 0, tune_polys: int = 0,
                    order: int = 0, log2_radix: int = 0, word_bits: int = 0, r1: int = 0, wg_size: int = 0,
                    col_width: int = 0) -> Plan:
    primes = [int(q) for q in primes]
    arr = (ctypes.c_uint64 * len(primes))(*primes)
    opts = _Opts(twiddle_mode, ot_stages, ot_log2_base, log2_n1, kernel_path, int(use_autotune), int(tune_polys),
                 int(order), int(log2_radix), int(word_bits), int(r1), int(wg_size), int(col_width))
    h = _vp()
    _check(_lib.ntt_plan_create(ctypes.byref(h), N, arr, len(primes), ctypes.byref(opts)), "ntt_plan_create")
    return Plan(h.value, N, len(primes))


def ntt_plan_destroy(plan: Plan) -> None:
    plan.destroy()


def ntt_plan_get_roots(plan: Plan) -> list[int]:
    out = (ctypes.c_uint64 * plan.L)()
    _check(_lib.ntt_plan_get_roots(plan.handle, out), "ntt_plan_get_roots")
    return list(out)


def ntt_plan_get_info(plan: Plan) -> dict:
    N, L, n1 = _u32(), _u32(), _u32()
    mode, ots, path = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.ntt_plan_get_info(plan.handle, ctypes.byref(N), ctypes.byref(L), ctypes.byref(n1),
                                  ctypes.byref(mode), ctypes.byref(ots), ctypes.byref(path)), "ntt_plan_get_info")
    r1, wg, cw = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.ntt_plan_get_tiles(plan.handle, ctypes.byref(r1), ctypes.byref(wg), ctypes.byref(cw)),
           "ntt_plan_get_tiles")
    return {"N": N.value, "L": L.value, "log2_n1": n1.value, "twiddle_mode": mode.value, "ot_stages": ots.value,
            "kernel_path": path.value, "r1": r1.value, "wg_size": wg.value, "col_width": cw.value}


def ntt_forward(plan: Plan, data, n_polys: int | None = None, stream=None) -> None:
    n, (d,) = _batch_addrs(plan, [data], ["data"], n_polys)
    _check(_lib.ntt_forward(plan.handle, d, n, _stream(stream)), "ntt_forward")


def ntt_inverse(plan: Plan, data, n_polys: int | None = None, stream=None) -> None:
    n, (d,) = _batch_addrs(plan, [data], ["data"], n_polys)
    _check(_lib.ntt_inverse(plan.handle, d, n, _stream(stream)), "ntt_inverse")


def ntt_forward_pass(plan: Plan, data, pass_index: int, n_polys: int | None = None, stream=None) -> None:
    n, (d,) = _batch_addrs(plan, [data], ["data"], n_polys)
    _check(_lib.ntt_forward_pass(plan.handle, d, n, pass_index, _stream(stream)), "ntt_forward_pass")


def ntt_inverse_pass(plan: Plan, data, pass_index: int, n_polys: int | None = None, stream=None) -> None:
    n, (d,) = _batch_addrs(plan, [data], ["data"], n_polys)
    _check(_lib.ntt_inverse_pass(plan.handle, d, n, pass_index, _stream(stream)), "ntt_inverse_pass")


def ntt_plan_num_passes(plan: Plan) -> int:
    return int(_lib.ntt_plan_num_passes(plan.handle))


def ntt_plan_log2_radix(plan: Plan) -> int:
    """Stages per launch of a PATH_RADIX2 (1) or PATH_REGISTER plan; 0 for the other paths."""
    r = int(_lib.ntt_plan_log2_radix(plan.handle))
    if r < 0:
        raise NttError(-1, "ntt_plan_log2_radix")
    return r


def ntt_plan_order(plan: Plan) -> int:
    """ORDER_BITREV or ORDER_NATURAL: the slot order of the plan's NTT domain."""
    r = int(_lib.ntt_plan_order(plan.handle))
    if r < 0:
        raise NttError(-1, "ntt_plan_order")
    return r


def ntt_plan_tuned(plan: Plan) -> bool:
    """Whether the plan's options came from the tuner's file (use_autotune=1 found its shape)."""
    r = int(_lib.ntt_plan_tuned(plan.handle))
    if r < 0:
        raise NttError(-1, "ntt_plan_tuned")
    return bool(r)


def ntt_pointwise_mul(plan: Plan, a, b, c, n_polys: int | None = None, stream=None) -> None:
    n, (pa, pb, pc) = _batch_addrs(plan, [a, b, c], ["a", "b", "c"], n_polys)
    _check(_lib.ntt_pointwise_mul(plan.handle, pa, pb, pc, n, _stream(stream)), "ntt_pointwise_mul")


def ntt_polymul_negacyclic(plan: Plan, a, b, c, n_polys: int | None = None, stream=None) -> None:
    n, (pa, pb, pc) = _batch_addrs(plan, [a, b, c], ["a", "b", "c"], n_polys)
    _check(_lib.ntt_polymul_negacyclic(plan.handle, pa, pb, pc, n, _stream(stream)), "ntt_polymul_negacyclic")


def ntt_polymul_negacyclic_noalloc(plan: Plan, a, b, c, n_polys: int | None = None, stream=None) -> None:
    """ntt_polymul_negacyclic with NTT(b) in the library's fixed device array: allocates
    nothing; at most ntt_polymul_noalloc_max_words() residues per call; calls that overlap
    on one device race."""
    n, (pa, pb, pc) = _batch_addrs(plan, [a, b, c], ["a", "b", "c"], n_polys)
    _check(_lib.ntt_polymul_negacyclic_noalloc(plan.handle, pa, pb, pc, n, _stream(stream)),
           "ntt_polymul_negacyclic_noalloc")


def ntt_polymul_noalloc_max_words() -> int:
    return int(_lib.ntt_polymul_noalloc_max_words())


# ---------------------------------------------------------------- 32-bit words
# Plans created with word_bits=32 (primes below 2^30) take [n_polys][L][N] tensors of 4-byte
# integers (int32 or uint32) through these calls.

def ntt_forward_u32(plan: Plan, data, n_polys: int | None = None, stream=None) -> None:
    n, (d,) = _batch_addrs(plan, [data], ["data"], n_polys, 4)
    _check(_lib.ntt_forward_u32(plan.handle, d, n, _stream(stream)), "ntt_forward_u32")


def ntt_inverse_u32(plan: Plan, data, n_polys: int | None = None, stream=None) -> None:
    n, (d,) = _batch_addrs(plan, [data], ["data"], n_polys, 4)
    _check(_lib.ntt_inverse_u32(plan.handle, d, n, _stream(stream)), "ntt_inverse_u32")


def ntt_pointwise_mul_u32(plan: Plan, a, b, c, n_polys: int | None = None, stream=None) -> None:
    n, (pa, pb, pc) = _batch_addrs(plan, [a, b, c], ["a", "b", "c"], n_polys, 4)
    _check(_lib.ntt_pointwise_mul_u32(plan.handle, pa, pb, pc, n, _stream(stream)), "ntt_pointwise_mul_u32")


def ntt_polymul_negacyclic_u32(plan: Plan, a, b, c, n_polys: int | None = None, stream=None) -> None:
    n, (pa, pb, pc) = _batch_addrs(plan, [a, b, c], ["a", "b", "c"], n_polys, 4)
    _check(_lib.ntt_polymul_negacyclic_u32(plan.handle, pa, pb, pc, n, _stream(stream)),
           "ntt_polymul_negacyclic_u32")


def ntt_plan_word_bits(plan: Plan) -> int:
    r = int(_lib.ntt_plan_word_bits(plan.handle))
    if r < 0:
        raise NttError(-1, "ntt_plan_word_bits")
    return r


# ---------------------------------------------------------------- RNS <-> integers
# Integers are [n_polys][W][N] int64/uint64 tensors of little-endian 64-bit words.

def ntt_crt_words(plan: Plan) -> int:
    """W: the 64-bit words of Q, the width of a reconstructed coefficient."""
    w = int(_lib.ntt_crt_words(plan.handle))
    if w == 0:
        raise NttError(-1, "ntt_crt_words")
    return w


def ntt_rns_decompose(plan: Plan, words, n_words: int, res, n_polys: int | None = None, stream=None) -> None:
    if n_polys is None:
        if isinstance(words, int):
            raise ValueError("n_polys is required when a buffer is given as a raw address")
        n_polys = words.numel() // (int(n_words) * plan.N)
    n_polys = int(n_polys)
    if n_polys < 1:
        raise ValueError("n_polys must be at least 1")
    pw = _addr(words, n_polys * int(n_words) * plan.N, "words")
    pr = _addr(res, n_polys * plan.L * plan.N, "res")
    _check(_lib.ntt_rns_decompose(plan.handle, pw, int(n_words), pr, n_polys, _stream(stream)), "ntt_rns_decompose")


def ntt_crt_reconstruct(plan: Plan, res, words, n_polys: int | None = None, stream=None) -> None:
    n, (pr,) = _batch_addrs(plan, [res], ["res"], n_polys)
    pw = _addr(words, n * ntt_crt_words(plan) * plan.N, "words")
    _check(_lib.ntt_crt_reconstruct(plan.handle, pr, pw, n, _stream(stream)), "ntt_crt_reconstruct")


class Batch:
    """Owns an ntt_batch_t.  Keeps the plans (and buffers passed as tensors) of its jobs alive."""

    def __init__(self, handle: int, keep):
        self.handle = handle
        self._keep = keep

    def destroy(self) -> None:
        if self.handle:
            _check(_lib.ntt_batch_destroy(self.handle), "ntt_batch_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _jobs_array(jobs):
    jobs = list(jobs)
    arr = (_Job * len(jobs))()
    keep = []
    for i, job in enumerate(jobs):
        plan, data, n_polys, n_limbs, op = job[:5]
        key = job[5] if len(job) > 5 else None
        limbs = n_limbs or plan.L
        if n_polys is None:
            if isinstance(data, int):
                raise ValueError(f"job {i}: n_polys is required when data is a raw address")
            n_polys = data.numel() // (plan.N * limbs)
        if int(n_polys) < 1:
            raise ValueError(f"job {i}: n_polys must be at least 1")
        d = _addr(data, int(n_polys) * limbs * plan.N, f"job {i} data")
        k = _addr(key, limbs * plan.N, f"job {i} key") if key is not None else None
        arr[i] = _Job(plan.handle, d, int(n_polys), int(n_limbs), int(op), 0, k)
        keep.append((plan, data, key))
    return arr, keep


def ntt_batch_assign(batch: "Batch", jobs, stream=None) -> None:
    """Replace the jobs of `batch`; descriptors are uploaded on `stream` (runs must follow there)."""
    arr, keep = _jobs_array(jobs)
    _check(_lib.ntt_batch_assign(batch.handle, arr, len(keep), _stream(stream)), "ntt_batch_assign")
    batch._keep = keep


def ntt_batch_create(jobs) -> Batch:
    """jobs: iterable of (plan, data, n_polys, n_limbs, op) or (plan, data, n_polys, n_limbs, op, key);
    n_polys None = from data's size, n_limbs 0 = all of the plan's primes, key = the NTT-domain
    [n_limbs][N] array multiplied in when op has OP_MULKEY."""
    arr, keep = _jobs_array(jobs)
    h = _vp()
    _check(_lib.ntt_batch_create(ctypes.byref(h), arr, len(keep)), "ntt_batch_create")
    return Batch(h.value, keep)


def ntt_batch_run(batch: Batch, mode: int = BATCH_GRAPH, stream=None) -> None:
    _check(_lib.ntt_batch_run(batch.handle, int(mode), _stream(stream)), "ntt_batch_run")


def ntt_batch_destroy(batch: Batch) -> None:
    batch.destroy()
