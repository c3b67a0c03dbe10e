"""Python binding of the C ABI in ``include/ct.h`` (argument marshalling only).

Every operation runs in the HIP library ``libct.so``; this module only turns torch tensors into
device pointers and the current torch stream into the ``hipStream_t`` the library enqueues on.
If the library is missing the import of a table or pool fails loudly: there is no fallback.

Keys are ``torch.int64`` tensors holding the u64 bit patterns.  32-bit values travel as
``torch.int32`` holding u32 bits, 64-bit values as ``torch.int64`` holding u64 bits.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libct.so")

CT_OK, CT_E_INVALID, CT_E_FULL, CT_E_EMPTY, CT_E_NOMEM, CT_E_HIP = range(6)
PRESENT, INSERTED, FULL = 0, 1, 2
ERR_FULL, ERR_POOL = 1, 2
KERNELS = ["clear", "prologue", "dedup", "insert", "erase", "apply", "rank", "final", "fix", "find"]
VAL_NONE, VAL_U32, VAL_U64 = 0, 1, 2
GROUP_MERGE_RUNS = 1
GROUP_BLOCK = {128: 7 << 8, 256: 0, 512: 9 << 8, 1024: 10 << 8}   # CT_GROUP_BLOCK(threads)
OP_CLEAR, OP_INSERT, OP_FIND, OP_ERASE = 0, 1, 2, 3
HASH_MIX64, HASH_VOXEL21 = 0, 1
INSERT_AUTO, INSERT_RESOLVE_FIRST, INSERT_SPECULATIVE = 0, 1, 2  # ct_table_set_insert_path
CHECK_SIZE, CHECK_DUPLICATE, CHECK_REACH, CHECK_POOL = 1, 2, 12, 32


class CtError(RuntimeError):
    pass


class TableDesc(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("val_kind", C.c_int32), ("hash_kind", C.c_int32),
                ("bucket_count", C.c_int64), ("chunk", C.c_int64)]


class ServerDesc(C.Structure):
    _fields_ = [("streams", C.c_int32), ("max_inflight", C.c_int32), ("max_batch_keys", C.c_int64)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("batches", C.c_int64),
                ("peak_staging_bytes", C.c_int64), ("peak_inflight", C.c_int64),
                ("dispatch_ns", C.c_int64), ("retire_ns", C.c_int64), ("error", C.c_int32)]


_lib = None

# name -> (restype, argtypes)
_P, _I64, _I32 = C.c_void_p, C.c_int64, C.c_int32
_PI64 = C.POINTER(C.c_int64)
SIGNATURES = {
    "ct_status_str": (C.c_char_p, [C.c_int]),
    "ct_table_bytes": (C.c_int, [C.POINTER(TableDesc), _PI64]),
    "ct_table_init": (C.c_int, [_P, _I64, C.POINTER(TableDesc), _P, C.POINTER(_P)]),
    "ct_table_destroy": (C.c_int, [_P]),
    "ct_table_info": (C.c_int, [_P, _PI64, _PI64]),
    "ct_table_set_profiling": (C.c_int, [_P, C.c_int]),
    "ct_table_profile": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_double), _PI64]),
    "ct_table_profile_reset": (C.c_int, [_P]),
    "ct_insert_batch": (C.c_int, [_P, _P, _P, _I64, _P, _P]),
    "ct_insert_batch_noalloc": (C.c_int, [_P, _P, _P, _I64, _P, _P]),
    "ct_find_batch": (C.c_int, [_P, _P, _I64, _P, _P, _P]),
    "ct_erase_batch": (C.c_int, [_P, _P, _I64, _P, _P]),
    "ct_size": (C.c_int, [_P, _PI64, _P]),
    "ct_clear": (C.c_int, [_P, _P]),
    "ct_dump": (C.c_int, [_P, _P, _P, _I64, _PI64, _P]),
    "ct_check_invariants": (C.c_int, [_P, _P, _PI64, _P]),
    "ct_check_invariants_detail": (C.c_int, [_P, _P, _PI64, C.POINTER(C.c_uint32), _P]),
    "ct_get_error": (C.c_int, [_P, C.POINTER(C.c_uint32), _P]),
    "ct_table_dedup_skewed": (C.c_int, [_P, C.POINTER(C.c_int32), _P]),
    "ct_table_set_insert_path": (C.c_int, [_P, _I32]),
    "ct_table_debug_inject_claim_losses": (C.c_int, [_P, C.c_uint32, _P]),
    "ct_table_rehash": (C.c_int, [_P, _P, _P]),
    "ct_table_health": (C.c_int, [_P, _PI64, _PI64, _P]),
    "ct_table_purge": (C.c_int, [_P, _P]),
    "ct_table_device_view": (C.c_int, [_P, _I32, _P, _I64]),
    "ct_dev_apply": (C.c_int, [_P, _I32, _P, _P, _I64, _P, _P, _P]),
    "ct_dev_apply_mixed": (C.c_int, [_P, _P, _P, _P, _I64, _P, _P, _P]),
    "ct_voxel_insert_neighbours": (C.c_int, [_P, _P, _I64, _I32, _P]),
    "ct_voxel_insert_neighbours_alloc": (C.c_int, [_P, _P, _P, _I64, _I32, _P]),
    "ct_pool_device_view": (C.c_int, [_P, _P, _I64]),
    "ct_dev_update_set": (C.c_int, [_P, _P, _P, _I64, _P, _P]),
    "ct_dev_pool_apply": (C.c_int, [_P, _I32, _P, _I64, _P, _P, _P]),
    "ct_select_key_range": (C.c_int, [_P, C.c_uint64, C.c_uint64, _P, _P, _I64, _PI64, _P]),
    "ct_select_voxel_box": (C.c_int, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), _P, _P,
                                      _I64, _PI64, _P]),
    "ct_pool_bytes": (C.c_int, [_I64, _PI64]),
    "ct_pool_init": (C.c_int, [_P, _I64, _I64, _P, C.POINTER(_P)]),
    "ct_pool_destroy": (C.c_int, [_P]),
    "ct_pool_pop_batch": (C.c_int, [_P, _I64, _P, _P, _P]),
    "ct_pool_push_batch": (C.c_int, [_P, _P, _I64, _P, _P]),
    "ct_pool_pop_front_batch": (C.c_int, [_P, _I64, _P, _P, _P]),
    "ct_pool_push_front_batch": (C.c_int, [_P, _P, _I64, _P, _P]),
    "ct_pool_size": (C.c_int, [_P, _PI64, _P]),
    "ct_pool_dump": (C.c_int, [_P, _P, _I64, _PI64, _P]),
    "ct_pool_get_error": (C.c_int, [_P, C.POINTER(C.c_uint32), _P]),
    "ct_insert_alloc_batch": (C.c_int, [_P, _P, _P, _I64, _P, _P, _P]),
    "ct_insert_alloc_batch_masked": (C.c_int, [_P, _P, _P, _P, _I64, _P, _P, _P]),
    "ct_erase_release_batch": (C.c_int, [_P, _P, _P, _I64, _P, _P]),
    "ct_plan_create": (C.c_int, [C.POINTER(_P)]),
    "ct_plan_destroy": (C.c_int, [_P]),
    "ct_plan_add": (C.c_int, [_P, _P, _I32, _P, _P, _P, _P, _I64]),
    "ct_plan_info": (C.c_int, [_P, _PI64, _PI64]),
    "ct_plan_launch": (C.c_int, [_P, _I32, _P]),
    "ct_plan_capture": (C.c_int, [_P, _I32, _P, C.POINTER(_P)]),
    "ct_plan_group_bytes": (C.c_int, [_P, _I32, _PI64]),
    "ct_plan_group": (C.c_int, [_P, _I32, _P, _I64]),
    "ct_plan_group_info": (C.c_int, [_P, _PI64, _PI64]),
    "ct_plan_launch_grouped": (C.c_int, [_P, _P]),
    "ct_plan_launch_single": (C.c_int, [_P, _I32, _P]),
    "ct_plan_capture_grouped": (C.c_int, [_P, _P, C.POINTER(_P)]),
    "ct_graph_launch": (C.c_int, [_P, _P]),
    "ct_graph_destroy": (C.c_int, [_P]),
    "ct_table_value_bytes": (C.c_int, [_P, C.POINTER(C.c_int32)]),
    "ct_server_create": (C.c_int, [C.POINTER(_P), _I32, C.POINTER(ServerDesc), _P, _I64,
                                   C.POINTER(_P)]),
    "ct_server_submit": (C.c_int, [_P, _I32, _I32, _P, _P, _I64, _P, _P, _PI64]),
    "ct_server_poll": (C.c_int, [_P, _P, _P, _P, _P, _I64, _PI64]),
    "ct_server_wait_idle": (C.c_int, [_P]),
    "ct_server_get_stats": (C.c_int, [_P, C.POINTER(ServerStats)]),
    "ct_server_now": (C.c_int, [_P, _PI64]),
    "ct_server_destroy": (C.c_int, [_P]),
    "ctr_gather": (C.c_int, [_P, _I64, _I32, _P, _I64, _P, _P]),
    "ctr_gather_cas": (C.c_int, [_P, _I64, _I32, _P, _I64, _P, _P]),
    "ctr_gather_cas_store": (C.c_int, [_P, _I64, _I32, _P, _I64, _P, _P]),
    "ctr_cas": (C.c_int, [_P, _I64, _P, _I64, _P]),
    "ctr_amin": (C.c_int, [_P, _I64, _P, _I64, _P]),
    "ctr_copy": (C.c_int, [_P, _P, _I64, _P]),
}


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise CtError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != CT_OK:
        msg = lib().ct_status_str(rc).decode()
        raise CtError(f"{what}: {msg} ({rc})")


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _need(t, dtype, n, name, device):
    if t.dtype != dtype:
        raise CtError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device != device:
        raise CtError(f"{name} must be on {device}")
    if not t.is_contiguous():
        raise CtError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise CtError(f"{name} must have {n} elements")


_VAL_DTYPE = {VAL_U32: torch.int32, VAL_U64: torch.int64}


class Pool:
    """Device index pool: a fixed-capacity int32 deque (back operations: the stack that feeds
    insert_alloc; front operations: pop_front / push_front)."""

    def __init__(self, capacity: int, device="cuda"):
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.capacity = int(capacity)
        nb = C.c_int64(0)
        _check(lib().ct_pool_bytes(self.capacity, C.byref(nb)), "ct_pool_bytes")
        self.buf = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        _check(lib().ct_pool_init(_ptr(self.buf), nb.value, self.capacity, _stream(self.device),
                                  C.byref(h)), "ct_pool_init")
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ct_pool_destroy(self._h)
            self._h = None

    def pop(self, n: int):
        out = torch.empty(int(n), dtype=torch.int32, device=self.device)
        st = torch.empty(int(n), dtype=torch.uint8, device=self.device)
        _check(lib().ct_pool_pop_batch(self._h, int(n), _ptr(out), _ptr(st), _stream(self.device)),
               "ct_pool_pop_batch")
        return out, st

    def push(self, values: torch.Tensor):
        _need(values, torch.int32, None, "values", self.device)
        st = torch.empty(values.numel(), dtype=torch.uint8, device=self.device)
        _check(lib().ct_pool_push_batch(self._h, _ptr(values), values.numel(), _ptr(st),
                                        _stream(self.device)), "ct_pool_push_batch")
        return st

    def pop_front(self, n: int):
        """pop_front n times (deque front operation): (values or -1, statuses)."""
        out = torch.empty(int(n), dtype=torch.int32, device=self.device)
        st = torch.empty(int(n), dtype=torch.uint8, device=self.device)
        _check(lib().ct_pool_pop_front_batch(self._h, int(n), _ptr(out), _ptr(st),
                                             _stream(self.device)), "ct_pool_pop_front_batch")
        return out, st

    def push_front(self, values: torch.Tensor):
        """push_front each value in order (the last ends up first): statuses."""
        _need(values, torch.int32, None, "values", self.device)
        st = torch.empty(values.numel(), dtype=torch.uint8, device=self.device)
        _check(lib().ct_pool_push_front_batch(self._h, _ptr(values), values.numel(), _ptr(st),
                                              _stream(self.device)), "ct_pool_push_front_batch")
        return st

    def dev_push_back(self, values: torch.Tensor):
        """push_back of every value by its own thread, concurrently (device-side API)."""
        _need(values, torch.int32, None, "values", self.device)
        st = torch.empty(values.numel(), dtype=torch.uint8, device=self.device)
        _check(lib().ct_dev_pool_apply(self._h, 0, _ptr(values), values.numel(), None, _ptr(st),
                                       _stream(self.device)), "ct_dev_pool_apply")
        return st

    def dev_pop_back(self, n: int):
        """n concurrent pop_back calls (device-side API): (values or -1, statuses)."""
        out = torch.empty(int(n), dtype=torch.int32, device=self.device)
        st = torch.empty(int(n), dtype=torch.uint8, device=self.device)
        _check(lib().ct_dev_pool_apply(self._h, 1, None, int(n), _ptr(out), _ptr(st),
                                       _stream(self.device)), "ct_dev_pool_apply")
        return out, st

    def size(self) -> int:
        v = C.c_int64(0)
        _check(lib().ct_pool_size(self._h, C.byref(v), _stream(self.device)), "ct_pool_size")
        return v.value

    def dump(self) -> torch.Tensor:
        n = self.size()
        out = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        cnt = C.c_int64(0)
        _check(lib().ct_pool_dump(self._h, _ptr(out), n, C.byref(cnt), _stream(self.device)),
               "ct_pool_dump")
        return out[:cnt.value]

    def error(self) -> int:
        e = C.c_uint32(0)
        _check(lib().ct_pool_get_error(self._h, C.byref(e), _stream(self.device)), "ct_pool_get_error")
        return e.value


class Table:
    """unordered_map (value_kind VAL_U32 / VAL_U64) or unordered_set (VAL_NONE) on one GPU."""

    def __init__(self, capacity: int, value_kind: int = VAL_U64, hash_kind: int = HASH_MIX64,
                 bucket_count: int = 0, chunk: int = 0, device="cuda"):
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.desc = TableDesc(int(capacity), int(value_kind), int(hash_kind), int(bucket_count),
                              int(chunk))
        nb = C.c_int64(0)
        _check(lib().ct_table_bytes(C.byref(self.desc), C.byref(nb)), "ct_table_bytes")
        self.nbytes = nb.value
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        _check(lib().ct_table_init(_ptr(self.buf), self.nbytes, C.byref(self.desc),
                                   _stream(self.device), C.byref(h)), "ct_table_init")
        self._h = h
        b = C.c_int64(0)
        c = C.c_int64(0)
        _check(lib().ct_table_info(self._h, C.byref(b), C.byref(c)), "ct_table_info")
        self.bucket_count = b.value
        self.chunk = c.value
        self.capacity = int(capacity)
        self.value_kind = int(value_kind)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ct_table_destroy(self._h)
            self._h = None

    @property
    def value_dtype(self):
        return _VAL_DTYPE.get(self.value_kind)

    def insert(self, keys: torch.Tensor, vals: torch.Tensor | None = None, status: bool = True):
        n = keys.numel()
        _need(keys, torch.int64, None, "keys", self.device)
        if self.value_kind != VAL_NONE:
            if vals is None:
                raise CtError("values are required for a map")
            _need(vals, self.value_dtype, n, "vals", self.device)
        st = torch.empty(n, dtype=torch.uint8, device=self.device) if status else None
        _check(lib().ct_insert_batch(self._h, _ptr(keys), _ptr(vals) if self.value_kind else None,
                                     n, _ptr(st), _stream(self.device)), "ct_insert_batch")
        return st

    def find(self, keys: torch.Tensor, values: bool = True, found: bool = True, out=None,
             found_out=None):
        """ct_find_batch: (values or None, found flags or None); `out` / `found_out` are written
        in place when given (no allocation: the call can be captured into a HIP graph)."""
        n = keys.numel()
        _need(keys, torch.int64, None, "keys", self.device)
        v = None
        if values and self.value_kind != VAL_NONE:
            if out is not None:
                _need(out, self.value_dtype, n, "out", self.device)
            v = out if out is not None else torch.empty(n, dtype=self.value_dtype, device=self.device)
        f = None
        if found:
            if found_out is not None:
                _need(found_out, torch.uint8, n, "found_out", self.device)
            f = found_out if found_out is not None else torch.empty(n, dtype=torch.uint8, device=self.device)
        _check(lib().ct_find_batch(self._h, _ptr(keys), n, _ptr(v), _ptr(f), _stream(self.device)),
               "ct_find_batch")
        return v, f

    def erase(self, keys: torch.Tensor, status: bool = True):
        n = keys.numel()
        _need(keys, torch.int64, None, "keys", self.device)
        er = torch.empty(n, dtype=torch.uint8, device=self.device) if status else None
        _check(lib().ct_erase_batch(self._h, _ptr(keys), n, _ptr(er), _stream(self.device)),
               "ct_erase_batch")
        return er

    def insert_alloc(self, pool: Pool, keys: torch.Tensor):
        n = keys.numel()
        _need(keys, torch.int64, None, "keys", self.device)
        out = torch.empty(n, dtype=torch.int32, device=self.device)
        st = torch.empty(n, dtype=torch.uint8, device=self.device)
        _check(lib().ct_insert_alloc_batch(self._h, pool._h, _ptr(keys), n, _ptr(out), _ptr(st),
                                           _stream(self.device)), "ct_insert_alloc_batch")
        return out, st

    def insert_alloc_masked(self, pool: Pool, keys: torch.Tensor, skip: torch.Tensor,
                            out: torch.Tensor | None = None, status: torch.Tensor | None = None):
        """insert_alloc of the keys whose skip byte is 0 (e.g. the found flags of a find of the
        same keys); the outputs of skipped elements are left as they are in `out` / `status`."""
        n = keys.numel()
        _need(keys, torch.int64, None, "keys", self.device)
        _need(skip, torch.uint8, n, "skip", self.device)
        if out is None:
            out = torch.full((n,), -1, dtype=torch.int32, device=self.device)
        if status is None:
            status = torch.full((n,), 0xFF, dtype=torch.uint8, device=self.device)
        _check(lib().ct_insert_alloc_batch_masked(self._h, pool._h, _ptr(keys), _ptr(skip), n,
                                                  _ptr(out), _ptr(status), _stream(self.device)),
               "ct_insert_alloc_batch_masked")
        return out, status

    def erase_release(self, pool: Pool, keys: torch.Tensor):
        n = keys.numel()
        _need(keys, torch.int64, None, "keys", self.device)
        er = torch.empty(n, dtype=torch.uint8, device=self.device)
        _check(lib().ct_erase_release_batch(self._h, pool._h, _ptr(keys), n, _ptr(er),
                                            _stream(self.device)), "ct_erase_release_batch")
        return er

    def size(self) -> int:
        v = C.c_int64(0)
        _check(lib().ct_size(self._h, C.byref(v), _stream(self.device)), "ct_size")
        return v.value

    def __len__(self):
        return self.size()

    def clear(self):
        _check(lib().ct_clear(self._h, _stream(self.device)), "ct_clear")

    def dump(self):
        """Live (keys, values) in unspecified order; values as int64 holding the slot's u64."""
        n = self.size()
        k = torch.empty(max(n, 1), dtype=torch.int64, device=self.device)
        v = torch.empty(max(n, 1), dtype=torch.int64, device=self.device)
        cnt = C.c_int64(0)
        _check(lib().ct_dump(self._h, _ptr(k), _ptr(v), n, C.byref(cnt), _stream(self.device)),
               "ct_dump")
        m = cnt.value
        return k[:m], v[:m]

    def select_key_range(self, lo: int, hi: int):
        """Live (keys, values) with lo <= key < hi (unsigned), in unspecified order."""
        return self._select(lambda k, v, cap, cnt: lib().ct_select_key_range(
            self._h, int(lo) & (2**64 - 1), int(hi) & (2**64 - 1), k, v, cap, cnt,
            _stream(self.device)), "ct_select_key_range")

    def select_voxel_box(self, lo3, hi3):
        """Live (keys, values) whose packed block coordinates lie in [lo3, hi3] (inclusive)."""
        lo = (C.c_int32 * 3)(*[int(x) for x in lo3])
        hi = (C.c_int32 * 3)(*[int(x) for x in hi3])
        return self._select(lambda k, v, cap, cnt: lib().ct_select_voxel_box(
            self._h, lo, hi, k, v, cap, cnt, _stream(self.device)), "ct_select_voxel_box")

    def _select(self, call, what):
        cap = self.size()
        k = torch.empty(max(cap, 1), dtype=torch.int64, device=self.device)
        v = torch.empty(max(cap, 1), dtype=torch.int64, device=self.device)
        cnt = C.c_int64(0)
        _check(call(_ptr(k), _ptr(v), cap, C.byref(cnt)), what)
        m = min(cnt.value, cap)
        return k[:m], v[:m]

    def dev_apply(self, op: int, keys: torch.Tensor, vals: torch.Tensor | None = None):
        """Per-thread operations through the device-side API, all elements concurrently and in
        no particular order (OP_INSERT / OP_ERASE / OP_FIND).  Returns (status, values or None)."""
        n = keys.numel()
        _need(keys, torch.int64, None, "keys", self.device)
        if op == OP_INSERT and self.value_kind != VAL_NONE:
            if vals is None:
                raise CtError("values are required for a map")
            _need(vals, self.value_dtype, n, "vals", self.device)
        st = torch.empty(n, dtype=torch.uint8, device=self.device)
        out = None
        if op == OP_FIND and self.value_kind != VAL_NONE:
            out = torch.empty(n, dtype=self.value_dtype, device=self.device)
        _check(lib().ct_dev_apply(self._h, int(op), _ptr(keys),
                                  _ptr(vals) if op == OP_INSERT and self.value_kind else None, n,
                                  _ptr(out), _ptr(st), _stream(self.device)), "ct_dev_apply")
        return st, out

    def dev_apply_mixed(self, ops: torch.Tensor, keys: torch.Tensor,
                        vals: torch.Tensor | None = None):
        """Per-thread operations of mixed kinds in one kernel: element i does ops[i] (OP_INSERT /
        OP_FIND / OP_ERASE, uint8) on keys[i], all concurrently.  Returns (status, values or
        None); values hold found values at find elements and the sentinel elsewhere."""
        n = keys.numel()
        _need(keys, torch.int64, None, "keys", self.device)
        _need(ops, torch.uint8, n, "ops", self.device)
        if self.value_kind != VAL_NONE:
            if vals is None:
                raise CtError("values are required for a map")
            _need(vals, self.value_dtype, n, "vals", self.device)
        st = torch.empty(n, dtype=torch.uint8, device=self.device)
        out = None
        if self.value_kind != VAL_NONE:
            out = torch.empty(n, dtype=self.value_dtype, device=self.device)
        _check(lib().ct_dev_apply_mixed(self._h, _ptr(ops), _ptr(keys),
                                        _ptr(vals) if self.value_kind else None, n, _ptr(out),
                                        _ptr(st), _stream(self.device)), "ct_dev_apply_mixed")
        return st, out

    def dev_update_set(self, set_table: "Table", keys: torch.Tensor):
        """In one kernel, every key that this map holds (contains) is inserted into `set_table`
        (device-side insert, concurrently): per-element status, 255 where this map lacks it."""
        _need(keys, torch.int64, None, "keys", self.device)
        st = torch.empty(keys.numel(), dtype=torch.uint8, device=self.device)
        _check(lib().ct_dev_update_set(self._h, set_table._h, _ptr(keys), keys.numel(), _ptr(st),
                                       _stream(self.device)), "ct_dev_update_set")
        return st

    def insert_neighbours(self, blocks: torch.Tensor, ndirs: int = 6):
        """Neighbour update of a voxel-block map through the device-side API."""
        _need(blocks, torch.int64, None, "blocks", self.device)
        _check(lib().ct_voxel_insert_neighbours(self._h, _ptr(blocks), blocks.numel(), int(ndirs),
                                                _stream(self.device)),
               "ct_voxel_insert_neighbours")

    def insert_neighbours_alloc(self, pool: "Pool", blocks: torch.Tensor, ndirs: int = 6):
        """Neighbour update whose new blocks take pop_back() of `pool` as their value."""
        _need(blocks, torch.int64, None, "blocks", self.device)
        _check(lib().ct_voxel_insert_neighbours_alloc(self._h, pool._h, _ptr(blocks),
                                                      blocks.numel(), int(ndirs),
                                                      _stream(self.device)),
               "ct_voxel_insert_neighbours_alloc")

    def rehash_into(self, dst: "Table"):
        """Insert every live pair of this table into `dst` (same value kind, room for all of them;
        keys `dst` holds keep their value there)."""
        if dst.device != self.device:
            raise CtError("rehash_into: both tables must be on one device")
        _check(lib().ct_table_rehash(self._h, dst._h, _stream(self.device)), "ct_table_rehash")

    def resized(self, capacity: int, bucket_count: int = 0, chunk: int = 0) -> "Table":
        """A new table of `capacity` (same value and hash kind) holding this table's pairs: the
        host-side resize; this table is unchanged."""
        t = Table(capacity, self.value_kind, self.desc.hash_kind, bucket_count, chunk,
                  device=self.device)
        self.rehash_into(t)
        return t

    def snapshot(self):
        """(keys, values) of every live pair, as device tensors: restore() them into this or any
        table of the same value kind."""
        return self.dump()

    def restore(self, keys: torch.Tensor, vals: torch.Tensor | None):
        """Make this table hold exactly the pairs of a snapshot (keys distinct)."""
        self.clear()
        if keys.numel():
            self.insert(keys, None if self.value_kind == VAL_NONE else
                        vals.to(self.value_dtype) if vals is not None else None, status=False)

    def check(self, pool: "Pool | None" = None) -> int:
        """Invariant violations found on the device (0 = consistent); with `pool`, also that the
        pool and this table's values together hold every pool index once."""
        v = C.c_int64(0)
        _check(lib().ct_check_invariants(self._h, pool._h if pool is not None else None,
                                         C.byref(v), _stream(self.device)),
               "ct_check_invariants")
        return v.value

    def check_detail(self, pool: "Pool | None" = None):
        """(violations, CHECK_* bits of the failed invariants)."""
        v, w = C.c_int64(0), C.c_uint32(0)
        _check(lib().ct_check_invariants_detail(self._h, pool._h if pool is not None else None,
                                                C.byref(v), C.byref(w), _stream(self.device)),
               "ct_check_invariants_detail")
        return v.value, w.value

    def error(self) -> int:
        e = C.c_uint32(0)
        _check(lib().ct_get_error(self._h, C.byref(e), _stream(self.device)), "ct_get_error")
        return e.value

    def debug_inject_claim_losses(self, every: int):
        """Test hook: treat the first claim of every `every`-th chunk element as lost (0 = off)."""
        _check(lib().ct_table_debug_inject_claim_losses(self._h, int(every), _stream(self.device)),
               "ct_table_debug_inject_claim_losses")

    def health(self):
        """(buckets without an empty slot, tombstone slots)."""
        c, tb = C.c_int64(0), C.c_int64(0)
        _check(lib().ct_table_health(self._h, C.byref(c), C.byref(tb), _stream(self.device)),
               "ct_table_health")
        return c.value, tb.value

    def purge(self):
        """Turn the tombstones of every bucket no live key passes into empty slots."""
        _check(lib().ct_table_purge(self._h, _stream(self.device)), "ct_table_purge")

    def dedup_skewed(self) -> bool:
        """True when recent chunks overflowed the dedup bins, so large chunks fold each tile's
        repeated keys first (a diagnostic: results never depend on it)."""
        v = C.c_int32(0)
        _check(lib().ct_table_dedup_skewed(self._h, C.byref(v), _stream(self.device)),
               "ct_table_dedup_skewed")
        return bool(v.value)

    def set_insert_path(self, path: int):
        """INSERT_AUTO (the default), INSERT_RESOLVE_FIRST or INSERT_SPECULATIVE."""
        _check(lib().ct_table_set_insert_path(self._h, int(path)), "ct_table_set_insert_path")

    def profiling(self, enable: bool = True):
        _check(lib().ct_table_set_profiling(self._h, int(enable)), "ct_table_set_profiling")

    def profile(self) -> dict:
        """{kernel kind: (total ms, launches)} recorded since profiling was enabled or reset."""
        out = {}
        for k, name in enumerate(KERNELS):
            ms = C.c_double(0)
            n = C.c_int64(0)
            _check(lib().ct_table_profile(self._h, k, C.byref(ms), C.byref(n)), "ct_table_profile")
            out[name] = (ms.value, n.value)
        return out

    def profile_reset(self):
        _check(lib().ct_table_profile_reset(self._h), "ct_table_profile_reset")


class Plan:
    """A schedule of operations on many tables, replayed on forked streams (include/ct.h)."""

    def __init__(self, device="cuda"):
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        h = C.c_void_p()
        _check(lib().ct_plan_create(C.byref(h)), "ct_plan_create")
        self._h = h
        self._keep = []  # tensors and tables the plan points at
        self._graph = None

    def __del__(self):
        if getattr(self, "_graph", None) and _lib is not None:
            _lib.ct_graph_destroy(self._graph)
            self._graph = None
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ct_plan_destroy(self._h)
            self._h = None

    def add(self, table: Table, op: int, keys=None, vals=None, vals_out=None, flags_out=None):
        n = 0 if keys is None else keys.numel()
        for tns in (keys, vals, vals_out, flags_out):
            if tns is not None:
                self._keep.append(tns)
        _check(lib().ct_plan_add(self._h, table._h, int(op), _ptr(keys), _ptr(vals), _ptr(vals_out),
                                 _ptr(flags_out), n), "ct_plan_add")
        self._keep.append(table)

    def info(self):
        a, b = C.c_int64(0), C.c_int64(0)
        _check(lib().ct_plan_info(self._h, C.byref(a), C.byref(b)), "ct_plan_info")
        return a.value, b.value

    def launch(self, lanes: int = 4):
        _check(lib().ct_plan_launch(self._h, int(lanes), _stream(self.device)), "ct_plan_launch")

    def capture(self, lanes: int = 4, stream=None):
        """Capture one run into a HIP graph on `stream` (a torch stream, not the default one)."""
        s = stream or torch.cuda.Stream(self.device)
        g = C.c_void_p()
        _check(lib().ct_plan_capture(self._h, int(lanes), s.cuda_stream, C.byref(g)), "ct_plan_capture")
        if self._graph:
            lib().ct_graph_destroy(self._graph)
        self._graph = g
        self._graph_stream = s
        return g

    def replay(self, stream=None):
        s = stream or self._graph_stream
        _check(lib().ct_graph_launch(self._graph, s.cuda_stream), "ct_graph_launch")

    # grouped form: one launch per stage per level over all tables
    def group(self, merge_runs: bool = False, block: int = 256):
        """Build the grouped form (descriptor buffer allocated here, kept by the plan); `block` is
        the threads per block of its find / insert / erase stages (128, 256, 512 or 1024)."""
        if block not in GROUP_BLOCK:
            raise CtError(f"block must be one of {sorted(GROUP_BLOCK)}")
        opt = (GROUP_MERGE_RUNS if merge_runs else 0) | GROUP_BLOCK[block]
        nb = C.c_int64(0)
        _check(lib().ct_plan_group_bytes(self._h, opt, C.byref(nb)), "ct_plan_group_bytes")
        self._gbuf = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        _check(lib().ct_plan_group(self._h, opt, _ptr(self._gbuf), nb.value), "ct_plan_group")

    def group_info(self):
        a, b = C.c_int64(0), C.c_int64(0)
        _check(lib().ct_plan_group_info(self._h, C.byref(a), C.byref(b)), "ct_plan_group_info")
        return a.value, b.value

    def launch_grouped(self):
        _check(lib().ct_plan_launch_grouped(self._h, _stream(self.device)), "ct_plan_launch_grouped")

    def launch_single(self, max_blocks: int = 0):
        """The grouped form as one cooperative launch (grid barriers between stages); needs the
        default 256-thread stages.  max_blocks > 0 caps the grid."""
        _check(lib().ct_plan_launch_single(self._h, int(max_blocks), _stream(self.device)),
               "ct_plan_launch_single")

    def capture_grouped(self, stream=None):
        s = stream or torch.cuda.Stream(self.device)
        g = C.c_void_p()
        _check(lib().ct_plan_capture_grouped(self._h, s.cuda_stream, C.byref(g)),
               "ct_plan_capture_grouped")
        if self._graph:
            lib().ct_graph_destroy(self._graph)
        self._graph = g
        self._graph_stream = s
        return g


# --- request server (include/ct_server.h) -------------------------------------------------------
class NativeServer:
    """Handle of a ct_server over `tables`, with a device staging buffer of `staging_bytes`.

    Host arrays handed to ``submit`` must stay alive until their request is reported complete;
    the caller keeps them (this class only keeps the tables and the staging buffer alive)."""

    def __init__(self, tables, staging_bytes: int, streams: int = 8, max_inflight: int = 64,
                 max_batch_keys: int = 1 << 21, device="cuda"):
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.tables = list(tables)
        self.staging = torch.empty(int(staging_bytes), dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        arr = (C.c_void_p * len(self.tables))(*[t._h.value for t in self.tables])
        d = ServerDesc(int(streams), int(max_inflight), int(max_batch_keys))
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().ct_server_create(C.cast(arr, C.POINTER(C.c_void_p)), len(self.tables),
                                          C.byref(d), _ptr(self.staging), self.staging.numel(),
                                          C.byref(h)), "ct_server_create")
        self._h = h

    def close(self):
        """Wait for every submitted request, stop the worker and free the server."""
        if getattr(self, "_h", None) and _lib is not None:
            h, self._h = self._h, None
            _check(_lib.ct_server_destroy(h), "ct_server_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 -- never raise from a finaliser
            pass

    def submit(self, table: int, op: int, keys, vals=None, vals_out=None, flags_out=None) -> int:
        """Queue one request; the arrays are host tensors (pinned for asynchronous copies)."""
        n = keys.numel()
        for t in (keys, vals, vals_out, flags_out):
            if t is not None and (t.is_cuda or not t.is_contiguous()):
                raise CtError("server arrays must be contiguous host tensors")
        tk = C.c_int64(0)
        _check(lib().ct_server_submit(self._h, int(table), int(op), _ptr(keys), _ptr(vals), n,
                                      _ptr(vals_out), _ptr(flags_out), C.byref(tk)),
               "ct_server_submit")
        return tk.value

    def poll(self, max_items: int = 1 << 16):
        """Completed requests: (tickets, submit_ns, done_ns, status) numpy arrays."""
        import numpy as np
        t = np.empty(max_items, dtype=np.int64)
        a = np.empty(max_items, dtype=np.int64)
        d = np.empty(max_items, dtype=np.int64)
        st = np.empty(max_items, dtype=np.int32)
        cnt = C.c_int64(0)
        _check(lib().ct_server_poll(self._h, t.ctypes.data, a.ctypes.data, d.ctypes.data,
                                    st.ctypes.data, max_items, C.byref(cnt)), "ct_server_poll")
        k = cnt.value
        return t[:k], a[:k], d[:k], st[:k]

    def wait_idle(self):
        _check(lib().ct_server_wait_idle(self._h), "ct_server_wait_idle")

    def now_ns(self) -> int:
        v = C.c_int64(0)
        _check(lib().ct_server_now(self._h, C.byref(v)), "ct_server_now")
        return v.value

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().ct_server_get_stats(self._h, C.byref(st)), "ct_server_get_stats")
        return {name: getattr(st, name) for name, _ in ServerStats._fields_}


# --- measured ceilings (include/ct_roofline.h) ------------------------------------------------
def gather(lines: torch.Tensor, nlines: int, line_bytes: int, keys: torch.Tensor, out: torch.Tensor,
           cas: bool = False, store: bool = False):
    """ctr_gather, ctr_gather_cas (cas) or ctr_gather_cas_store (cas and store)."""
    f = (lib().ctr_gather_cas_store if store else lib().ctr_gather_cas) if cas else lib().ctr_gather
    _check(f(_ptr(lines), int(nlines), int(line_bytes), _ptr(keys), keys.numel(), _ptr(out),
             _stream(keys.device)), "ctr_gather")


def cas_words(words: torch.Tensor, nwords: int, keys: torch.Tensor):
    _check(lib().ctr_cas(_ptr(words), int(nwords), _ptr(keys), keys.numel(), _stream(keys.device)),
           "ctr_cas")


def amin_words(words: torch.Tensor, nwords: int, keys: torch.Tensor):
    _check(lib().ctr_amin(_ptr(words), int(nwords), _ptr(keys), keys.numel(), _stream(keys.device)),
           "ctr_amin")


def copy(src: torch.Tensor, dst: torch.Tensor, nbytes: int):
    _check(lib().ctr_copy(_ptr(src), _ptr(dst), int(nbytes), _stream(src.device)), "ctr_copy")
