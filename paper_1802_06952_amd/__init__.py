"""Python binding of libqs (ctypes): argument marshalling only.

Every step of the simulation runs in the HIP kernels of ``libqs.so``; this
module only converts Python/numpy arguments and raises on error codes.  The
library must have been built in-tree (``python -m paper_1802_06952_amd.build``);
importing fails loudly when it is missing.

The functions carry the names of the C ABI (``include/qs.h``):
``qs_load_circuit``, ``qs_partition``, ``qs_plan_info``, ``qs_plan_dump``,
``qs_run_halves``, ``qs_amplitudes`` and friends.  ``Plan`` wraps them.
"""

from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqs.so")

QS_OK = 0
QS_PREC_FP32 = 0
QS_PREC_SPLIT_BF16 = 1
_STATUS = {0: "QS_OK", -1: "QS_ERR_ARG", -2: "QS_ERR_PARSE", -3: "QS_ERR_UNSUPPORTED",
           -4: "QS_ERR_OOM", -5: "QS_ERR_HIP", -6: "QS_ERR_STATE"}

EXPORTED = ("qs_last_error", "qs_load_circuit", "qs_circuit_info", "qs_circuit_free",
            "qs_partition", "qs_plan_info", "qs_plan_dump", "qs_plan_free", "qs_run_halves",
            "qs_amplitudes", "qs_amplitudes_device", "qs_amplitudes_device_static", "qs_run_graph",
            "qs_half_amplitudes", "qs_plan_reset",
            "qs_get_timing", "qs_set_timing", "qs_get_pass_timing", "qs_score_cut", "qs_choose_cut",
            "qs_partition_chain", "qs_chain_info", "qs_chain_register", "qs_chain_amplitudes_device",
            "qs_chain_amplitudes", "qs_chain_free")


class QSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class qs_cut_score(C.Structure):
    _fields_ = [("n_cuts", C.c_int), ("n_upper", C.c_int), ("n_lower", C.c_int),
                ("equivalent_qubits", C.c_int), ("flat_updates", C.c_double),
                ("plan_cost", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class qs_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class qs_options(C.Structure):
    _fields_ = [("tile_bits", C.c_int), ("coalesce_bits", C.c_int), ("tail_max_qubits", C.c_int),
                ("materialize_level", C.c_int), ("plain", C.c_int), ("mem_budget", C.c_size_t),
                ("one_stream", C.c_int), ("copies_per_launch", C.c_uint64),
                ("max_stages", C.c_int), ("min_tile_bits", C.c_int), ("no_exchange", C.c_int),
                ("alloc", qs_allocator)]


class TorchAllocator:
    """qs_allocator backed by PyTorch's caching allocator (device memory of
    the current device).  Keeps the ctypes callbacks alive while a plan uses
    them; counts the calls (``n_alloc``, ``n_free``)."""

    def __init__(self):
        import torch
        self._torch = torch
        self.n_alloc = 0
        self.n_free = 0
        self.live = 0

        def _alloc(nbytes, _ctx):
            try:
                ptr = self._torch.cuda.caching_allocator_alloc(int(nbytes))
            except Exception:  # out of memory: the library reports QS_ERR_OOM
                return None
            self.n_alloc += 1
            self.live += 1
            return ptr

        def _free(ptr, _ctx):
            if ptr:
                self._torch.cuda.caching_allocator_delete(ptr)
                self.n_free += 1
                self.live -= 1

        self._alloc_cb = ALLOC_FN(_alloc)
        self._free_cb = FREE_FN(_free)
        self.struct = qs_allocator(self._alloc_cb, self._free_cb, None)


def _allocator(alloc):
    """None -> hipMalloc / hipFree inside the library; "torch" -> a new TorchAllocator."""
    if alloc is None:
        return None
    if alloc == "torch":
        return TorchAllocator()
    return alloc


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1802_06952_amd.build`")
    # torch ships its own HIP runtime; loaded first, it is the one the library
    # binds to (same soname).  Loading the library first would put a second
    # HIP/HSA runtime into a process that later imports torch, and device
    # allocations then fail.
    try:
        import torch  # noqa: F401
    except ImportError:  # pragma: no cover - torch is part of the image
        pass
    lib = C.CDLL(LIB_PATH)
    vp, u64p = C.c_void_p, C.POINTER(C.c_uint64)
    lib.qs_last_error.restype = C.c_char_p
    lib.qs_load_circuit.argtypes = [C.c_char_p, C.c_size_t, C.POINTER(vp)]
    lib.qs_circuit_info.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    lib.qs_circuit_free.argtypes = [vp]
    lib.qs_circuit_free.restype = None
    lib.qs_partition.argtypes = [vp, C.c_uint64, C.POINTER(qs_options), C.POINTER(vp)]
    lib.qs_plan_info.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
    lib.qs_score_cut.argtypes = [vp, C.c_uint64, C.c_int, C.POINTER(qs_cut_score)]
    lib.qs_choose_cut.argtypes = [vp, u64p, C.c_size_t, C.c_int, C.c_int,
                                  C.POINTER(C.c_size_t), C.POINTER(qs_cut_score)]
    lib.qs_plan_dump.argtypes = [vp, C.c_uint64, C.c_uint64, C.c_char_p, C.c_size_t,
                                 C.POINTER(C.c_size_t)]
    lib.qs_plan_free.argtypes = [vp]
    lib.qs_plan_free.restype = None
    lib.qs_run_halves.argtypes = [vp, C.c_uint64, C.c_uint64, u64p, C.c_size_t, vp]
    lib.qs_amplitudes.argtypes = [vp, u64p, C.c_size_t, C.c_int, C.POINTER(C.c_float),
                                  C.POINTER(C.c_double), vp]
    lib.qs_amplitudes_device.argtypes = [vp, C.c_int, vp, vp, vp]
    lib.qs_amplitudes_device_static.argtypes = [vp, C.c_int, vp, vp, vp]
    lib.qs_run_graph.argtypes = [vp, C.c_uint64, C.c_uint64, C.c_int, vp, vp, vp]
    lib.qs_half_amplitudes.argtypes = [vp, C.c_int, C.c_uint64, C.c_uint64, C.POINTER(C.c_float),
                                       C.c_size_t, C.POINTER(C.c_size_t), vp]
    lib.qs_plan_reset.argtypes = [vp, C.c_int]
    lib.qs_get_timing.argtypes = [vp, C.POINTER(C.c_double)]
    lib.qs_set_timing.argtypes = [vp, C.c_int]
    lib.qs_get_pass_timing.argtypes = [vp, C.POINTER(C.c_double), C.c_size_t,
                                       C.POINTER(C.c_size_t)]
    lib.qs_partition_chain.argtypes = [vp, u64p, C.c_int, C.POINTER(qs_options), C.POINTER(vp)]
    lib.qs_chain_info.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
    lib.qs_chain_register.argtypes = [vp, u64p, C.c_size_t]
    lib.qs_chain_amplitudes_device.argtypes = [vp, vp, vp, vp]
    lib.qs_chain_amplitudes.argtypes = [vp, u64p, C.c_size_t, C.POINTER(C.c_float),
                                        C.POINTER(C.c_double), vp]
    lib.qs_chain_free.argtypes = [vp]
    lib.qs_chain_free.restype = None
    for name in EXPORTED:
        if name != "qs_last_error" and getattr(lib, name).restype is not None:
            getattr(lib, name).restype = C.c_int
    return lib


_lib = _load()


def lib() -> C.CDLL:
    return _lib


def _check(status: int) -> None:
    if status != QS_OK:
        raise QSError(status, _lib.qs_last_error().decode())


def _stream_handle(stream) -> int | None:
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available() and torch.cuda.is_initialized():
                return torch.cuda.current_stream().cuda_stream
        except Exception:  # pragma: no cover - torch is optional here
            pass
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _bits(bitstrings) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(bitstrings, dtype=np.uint64))


# --------------------------------------------------------------- C ABI names

def qs_load_circuit(text: str) -> C.c_void_p:
    b = text.encode()
    h = C.c_void_p()
    _check(_lib.qs_load_circuit(b, len(b), C.byref(h)))
    return h


def qs_circuit_info(circ) -> tuple[int, int]:
    n, g = C.c_int(), C.c_int()
    _check(_lib.qs_circuit_info(circ, C.byref(n), C.byref(g)))
    return n.value, g.value


def qs_circuit_free(circ) -> None:
    _lib.qs_circuit_free(circ)


def qs_partition(circ, upper_mask: int, opts: qs_options | None = None) -> C.c_void_p:
    h = C.c_void_p()
    _check(_lib.qs_partition(circ, C.c_uint64(upper_mask), C.byref(opts) if opts else None,
                             C.byref(h)))
    return h


def qs_score_cut(circ, upper_mask: int, n_values: int) -> dict:
    sc = qs_cut_score()
    _check(_lib.qs_score_cut(circ, upper_mask, n_values, C.byref(sc)))
    return sc.as_dict()


def qs_choose_cut(circ, masks, n_values: int, criterion: int = 0) -> tuple[int, dict]:
    """Index of the best candidate mask (criterion 0: Eq. 2 flat updates, 1: plan cost) and its score."""
    arr = np.ascontiguousarray(np.asarray(masks, dtype=np.uint64))
    best = C.c_size_t()
    sc = qs_cut_score()
    _check(_lib.qs_choose_cut(circ, arr.ctypes.data_as(C.POINTER(C.c_uint64)), arr.size, n_values,
                              criterion, C.byref(best), C.byref(sc)))
    return best.value, sc.as_dict()


def qs_plan_info(plan) -> tuple[int, int, int]:
    a, b, c = C.c_int(), C.c_int(), C.c_int()
    _check(_lib.qs_plan_info(plan, C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def qs_plan_dump(plan, copy_begin: int = 0, copy_end: int | None = None) -> dict:
    """Plan of the first copy block of [copy_begin, copy_end) (default: all copies)."""
    if copy_end is None:
        copy_end = 1 << qs_plan_info(plan)[2]
    need = C.c_size_t()
    _check(_lib.qs_plan_dump(plan, copy_begin, copy_end, None, 0, C.byref(need)))
    buf = C.create_string_buffer(need.value)
    _check(_lib.qs_plan_dump(plan, copy_begin, copy_end, buf, need.value, C.byref(need)))
    return json.loads(buf.value.decode())


def qs_plan_free(plan) -> None:
    _lib.qs_plan_free(plan)


def qs_plan_reset(plan, keep_bitstrings: bool = False) -> None:
    _check(_lib.qs_plan_reset(plan, 1 if keep_bitstrings else 0))


def qs_run_halves(plan, copy_begin: int, copy_end: int, bitstrings=None, stream=None) -> None:
    """bitstrings=None runs with the registered set."""
    if bitstrings is None:
        _check(_lib.qs_run_halves(plan, copy_begin, copy_end, None, 0, _stream_handle(stream)))
        return
    b = _bits(bitstrings)
    _check(_lib.qs_run_halves(plan, copy_begin, copy_end,
                              b.ctypes.data_as(C.POINTER(C.c_uint64)), b.size,
                              _stream_handle(stream)))


def qs_amplitudes(plan, bitstrings, prec: int = QS_PREC_FP32, stream=None):
    """Returns (amplitudes as complex64 array, stats array of 3 float64)."""
    b = _bits(bitstrings)
    out = np.empty(2 * b.size, dtype=np.float32)
    stats = np.zeros(3, dtype=np.float64)
    _check(_lib.qs_amplitudes(plan, b.ctypes.data_as(C.POINTER(C.c_uint64)), b.size, prec,
                              out.ctypes.data_as(C.POINTER(C.c_float)),
                              stats.ctypes.data_as(C.POINTER(C.c_double)), _stream_handle(stream)))
    return out.view(np.complex64), stats


def qs_amplitudes_device(plan, prec: int, d_out_ptr: int, d_sums_ptr: int | None = None,
                         stream=None) -> None:
    """Device outputs (raw device pointers, e.g. torch tensor.data_ptr())."""
    _check(_lib.qs_amplitudes_device(plan, prec, C.c_void_p(d_out_ptr),
                                     C.c_void_p(d_sums_ptr) if d_sums_ptr else None,
                                     _stream_handle(stream)))


def qs_amplitudes_device_static(plan, prec: int, d_out_ptr: int, d_sums_ptr: int | None = None,
                                stream=None) -> None:
    """As qs_amplitudes_device, with the assembly's scratch in the library's
    static region (no allocation)."""
    _check(_lib.qs_amplitudes_device_static(plan, prec, C.c_void_p(d_out_ptr),
                                            C.c_void_p(d_sums_ptr) if d_sums_ptr else None,
                                            _stream_handle(stream)))


def qs_run_graph(plan, copy_begin: int, copy_end: int, prec: int, d_out_ptr: int,
                 d_sums_ptr: int | None = None, stream=None) -> None:
    _check(_lib.qs_run_graph(plan, copy_begin, copy_end, prec, C.c_void_p(d_out_ptr),
                             C.c_void_p(d_sums_ptr) if d_sums_ptr else None, _stream_handle(stream)))


def qs_half_amplitudes(plan, side: int, copy_begin: int, copy_end: int, n_values: int,
                       stream=None) -> np.ndarray:
    """Per-copy half amplitudes [copy][value] of a run copy block (complex64)."""
    out = np.empty(2 * (copy_end - copy_begin) * n_values, dtype=np.float32)
    nv = C.c_size_t()
    _check(_lib.qs_half_amplitudes(plan, side, copy_begin, copy_end,
                                   out.ctypes.data_as(C.POINTER(C.c_float)), out.size // 2,
                                   C.byref(nv), _stream_handle(stream)))
    return out.view(np.complex64).reshape(copy_end - copy_begin, nv.value)


def qs_set_timing(plan, enable) -> None:
    """enable: False/0 off, True/1 per kernel family, 2 also per full-state pass."""
    _check(_lib.qs_set_timing(plan, int(enable)))


PASS_TIMING_FIELDS = ("side", "pass", "level_in", "stages", "tiles", "bytes", "ms", "passes")


def qs_get_pass_timing(plan) -> list[dict]:
    n = C.c_size_t(0)
    _check(_lib.qs_get_pass_timing(plan, None, 0, C.byref(n)))
    nf = len(PASS_TIMING_FIELDS)
    out = np.zeros(nf * max(1, n.value), dtype=np.float64)
    _check(_lib.qs_get_pass_timing(plan, out.ctypes.data_as(C.POINTER(C.c_double)), n.value,
                                   C.byref(n)))
    recs = []
    for r in out[: nf * n.value].reshape(-1, nf):
        d = dict(zip(PASS_TIMING_FIELDS, r.tolist()))
        for k in ("side", "pass", "level_in", "stages", "tiles", "passes"):
            d[k] = int(d[k])
        recs.append(d)
    return recs


TIMING_FIELDS = ("pass_ms", "tail_ms", "gemm_ms", "other_ms", "pass_launches", "tail_launches",
                 "gemm_launches", "other_launches", "pass_bytes", "gemm_flops", "tail_flops")


def qs_get_timing(plan) -> dict:
    out = np.zeros(11, dtype=np.float64)
    _check(_lib.qs_get_timing(plan, out.ctypes.data_as(C.POINTER(C.c_double))))
    return dict(zip(TIMING_FIELDS, out.tolist()))


def qs_partition_chain(circ, part_masks, opts: qs_options | None = None) -> C.c_void_p:
    masks = np.ascontiguousarray(np.asarray(part_masks, dtype=np.uint64))
    out = C.c_void_p()
    _check(_lib.qs_partition_chain(circ, masks.ctypes.data_as(C.POINTER(C.c_uint64)), masks.size,
                                   C.byref(opts) if opts is not None else None, C.byref(out)))
    return out


def qs_chain_info(plan) -> tuple[int, list[int], list[int]]:
    t = C.c_int()
    _check(_lib.qs_chain_info(plan, C.byref(t), None, None))
    pq = (C.c_int * t.value)()
    lc = (C.c_int * max(1, t.value - 1))()
    _check(_lib.qs_chain_info(plan, None, pq, lc))
    return t.value, list(pq), list(lc)[: t.value - 1]


def qs_chain_register(plan, bitstrings) -> None:
    b = _bits(bitstrings)
    _check(_lib.qs_chain_register(plan, b.ctypes.data_as(C.POINTER(C.c_uint64)), b.size))


def qs_chain_amplitudes_device(plan, d_out_ptr: int, d_sums_ptr: int | None = None,
                               stream=None) -> None:
    _check(_lib.qs_chain_amplitudes_device(plan, C.c_void_p(d_out_ptr),
                                           C.c_void_p(d_sums_ptr) if d_sums_ptr else None,
                                           _stream_handle(stream)))


def qs_chain_amplitudes(plan, bitstrings, stream=None):
    """Returns (amplitudes as complex64 array, stats array of 3 float64)."""
    b = _bits(bitstrings)
    out = np.empty(2 * b.size, dtype=np.float32)
    stats = np.zeros(3, dtype=np.float64)
    _check(_lib.qs_chain_amplitudes(plan, b.ctypes.data_as(C.POINTER(C.c_uint64)), b.size,
                                    out.ctypes.data_as(C.POINTER(C.c_float)),
                                    stats.ctypes.data_as(C.POINTER(C.c_double)),
                                    _stream_handle(stream)))
    return out.view(np.complex64), stats


def qs_chain_free(plan) -> None:
    _lib.qs_chain_free(plan)


# --------------------------------------------------------------- convenience


class ChainPlan:
    """Owns a circuit handle and a chain-partition plan (t parts)."""

    def __init__(self, circuit_text: str, part_masks, tile_bits: int = 0, tail_max_qubits: int = 0,
                 materialize_level: int = -1, mem_budget: int = 0, alloc="torch"):
        self.allocator = _allocator(alloc)
        self._circ = qs_load_circuit(circuit_text)
        opts = qs_options(tile_bits, 0, tail_max_qubits, materialize_level, 0, mem_budget, 1)
        if self.allocator is not None:
            opts.alloc = self.allocator.struct
        try:
            self._plan = qs_partition_chain(self._circ, part_masks, opts)
        except Exception:
            qs_circuit_free(self._circ)
            self._circ = None  # close() must not free it again
            raise
        self.t, self.part_qubits, self.link_cuts = qs_chain_info(self._plan)

    def register(self, bitstrings) -> None:
        qs_chain_register(self._plan, bitstrings)

    def amplitudes(self, bitstrings, stream=None):
        return qs_chain_amplitudes(self._plan, bitstrings, stream)

    def amplitudes_device(self, d_out_ptr: int, d_sums_ptr: int | None = None, stream=None) -> None:
        qs_chain_amplitudes_device(self._plan, d_out_ptr, d_sums_ptr, stream)

    def close(self) -> None:
        if getattr(self, "_plan", None):
            qs_chain_free(self._plan)
            self._plan = None
        if getattr(self, "_circ", None):
            qs_circuit_free(self._circ)
            self._circ = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

class Plan:
    """Owns a circuit handle and a plan handle.

    ``alloc``: "torch" (default) routes the plan's device memory through
    PyTorch's caching allocator; None lets the library call hipMalloc; any
    object with a ``struct`` attribute (a ``qs_allocator``) is passed as is.
    """

    def __init__(self, circuit_text: str, upper_mask: int, tile_bits: int = 0,
                 coalesce_bits: int = 0, tail_max_qubits: int = 0, materialize_level: int = -1,
                 plain: bool = False, mem_budget: int = 0, one_stream: bool = False,
                 copies_per_launch: int = 0, max_stages: int = 0, min_tile_bits: int = 0,
                 no_exchange: bool = False, alloc="torch"):
        self.allocator = _allocator(alloc)
        self._circ = qs_load_circuit(circuit_text)
        opts = qs_options(tile_bits, coalesce_bits, tail_max_qubits, materialize_level,
                          1 if plain else 0, mem_budget, 1 if one_stream else 0, copies_per_launch,
                          max_stages, min_tile_bits, 1 if no_exchange else 0)
        if self.allocator is not None:
            opts.alloc = self.allocator.struct
        try:
            self._plan = qs_partition(self._circ, upper_mask, opts)
        except Exception:
            qs_circuit_free(self._circ)
            self._circ = None  # close() must not free it again
            raise
        self.n_upper, self.n_lower, self.n_cuts = qs_plan_info(self._plan)

    @property
    def handle(self):
        return self._plan

    def dump(self, copy_begin: int = 0, copy_end: int | None = None) -> dict:
        return qs_plan_dump(self._plan, copy_begin, copy_end)

    def run_halves(self, copy_begin: int, copy_end: int, bitstrings=None, stream=None) -> None:
        qs_run_halves(self._plan, copy_begin, copy_end, bitstrings, stream)

    def amplitudes(self, bitstrings, prec: int = QS_PREC_FP32, stream=None):
        return qs_amplitudes(self._plan, bitstrings, prec, stream)

    def amplitudes_device(self, prec: int, d_out_ptr: int, d_sums_ptr: int | None = None,
                          stream=None) -> None:
        qs_amplitudes_device(self._plan, prec, d_out_ptr, d_sums_ptr, stream)

    def amplitudes_device_static(self, prec: int, d_out_ptr: int, d_sums_ptr: int | None = None,
                                 stream=None) -> None:
        qs_amplitudes_device_static(self._plan, prec, d_out_ptr, d_sums_ptr, stream)

    def run_graph(self, copy_begin: int, copy_end: int, prec: int, d_out_ptr: int,
                  d_sums_ptr: int | None = None, stream=None) -> None:
        qs_run_graph(self._plan, copy_begin, copy_end, prec, d_out_ptr, d_sums_ptr, stream)

    def half_amplitudes(self, side: int, copy_begin: int, copy_end: int, n_values: int,
                        stream=None) -> np.ndarray:
        return qs_half_amplitudes(self._plan, side, copy_begin, copy_end, n_values, stream)

    def reset(self, keep_bitstrings: bool = False) -> None:
        qs_plan_reset(self._plan, keep_bitstrings)

    def set_timing(self, on) -> None:
        qs_set_timing(self._plan, on)

    def timing(self) -> dict:
        return qs_get_timing(self._plan)

    def pass_timing(self) -> list[dict]:
        return qs_get_pass_timing(self._plan)

    def close(self) -> None:
        if getattr(self, "_plan", None):
            qs_plan_free(self._plan)
            self._plan = None
        if getattr(self, "_circ", None):
            qs_circuit_free(self._circ)
            self._circ = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
