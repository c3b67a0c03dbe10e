"""CPU oracle for the batch container operations -- TEST INFRASTRUCTURE.

A thin ctypes wrapper over ``oracle.c`` (plain sequential replay over a chained hash map and
LIFO stacks; see that file's header for the semantics and the paper passages they follow).
Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this package.
It shares no code with the GPU library, and the GPU library never imports it.

Parity status of each function (what pins it is in the test suite):
  insert / find / erase / size / clear / dump   pinned: brute force, dict replay, invariants
  insert_alloc / erase_release / pool ops      pinned: brute force, closed-form pool order
  voxel21 hash                                 pinned: the paper's printed constants, XOR
                                               decomposition, 21-bit field independence
  mix64 hash                                   decides bucket membership only; results do not
                                               depend on it (checked by a hash-swap test)
  partitioned multi-core replay                timing baseline only; checked equal to the
                                               sequential replay (per-key independence)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SRC_PART = os.path.join(_HERE, "partitioned.c")
_LIB = os.path.join(_HERE, "liboracle.so")

PRESENT, INSERTED, FULL = 0, 1, 2
HASH_MIX64, HASH_VOXEL21 = 0, 1

_lib = None


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc into ``liboracle.so`` next to it."""
    if force or not os.path.exists(_LIB):
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", _SRC,
                               _SRC_PART, "-o", _LIB])
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        P, I64, U64, I = C.c_void_p, C.c_int64, C.c_uint64, C.c_int
        sig = {
            "or_fmix64": (U64, [U64]),
            "or_voxel21_hash": (U64, [U64]),
            "or_bucket_of": (I64, [P, U64]),
            "or_table_new": (P, [I64, I, I64]),
            "or_table_free": (None, [P]),
            "or_size": (I64, [P]),
            "or_error": (I, [P]),
            "or_clear": (None, [P]),
            "or_insert": (None, [P, P, P, I64, P]),
            "or_find": (None, [P, P, I64, P, U64, P]),
            "or_erase": (None, [P, P, I64, P]),
            "or_pool_new": (P, [I64]),
            "or_pool_free": (None, [P]),
            "or_pool_size": (I64, [P]),
            "or_part_new": (P, [I64, I, C.c_double]),
            "or_part_free": (None, [P]),
            "or_part_size": (I64, [P]),
            "or_part_insert": (I, [P, P, P, I64, P]),
            "or_part_find": (I, [P, P, I64, P, U64, P]),
            "or_part_erase": (I, [P, P, I64, P]),
            "or_pool_dump": (I64, [P, P, I64]),
            "or_pool_pop": (None, [P, I64, P, P]),
            "or_pool_push": (None, [P, P, I64, P]),
            "or_pool_pop_front": (None, [P, I64, P, P]),
            "or_select": (I64, [P, C.c_int, C.c_uint64, C.c_uint64, P, P, P, P, I64]),
            "or_voxel_neighbour_keys": (I64, [P, I64, C.c_int, P]),
            "or_pool_push_front": (None, [P, P, I64, P]),
            "or_insert_alloc": (None, [P, P, P, I64, P, P]),
            "or_erase_release": (None, [P, P, P, I64, P]),
            "or_dump": (I64, [P, P, P, I64]),
            "or_check": (I64, [P, P, I, C.POINTER(C.c_int)]),
            "or_corrupt": (I, [P, P, I]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _u64(a):
    return np.ascontiguousarray(np.asarray(a).view(np.uint64) if np.asarray(a).dtype == np.int64
                                else np.asarray(a, dtype=np.uint64))


def voxel21_hash(key: int) -> int:
    """The spatial hash of a packed int3 key, as a 64-bit size_t (before the bucket reduction)."""
    return int(lib().or_voxel21_hash(int(key)))


def fmix64(key: int) -> int:
    return int(lib().or_fmix64(int(key)))


class PartitionedOracle:
    """Multi-core timing baseline: `parts` oracle tables, one thread each, keys split by hash
    (``partitioned.c``).  u64 values.  Results equal the sequential replay while no partition
    fills up (each gets `slack` times its share of the capacity)."""

    def __init__(self, capacity: int, parts: int, slack: float = 1.25):
        self.parts = int(parts)
        self._h = lib().or_part_new(int(capacity), self.parts, float(slack))
        if not self._h:
            raise MemoryError("partitioned oracle allocation failed")

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_part_free(self._h)
            self._h = None

    def size(self) -> int:
        return int(lib().or_part_size(self._h))

    def insert(self, keys, vals) -> np.ndarray:
        k, v = _u64(keys), _u64(vals)
        st = np.empty(k.size, dtype=np.uint8)
        if lib().or_part_insert(self._h, _ptr(k), _ptr(v), k.size, _ptr(st)):
            raise MemoryError("partitioned insert")
        return st

    def find(self, keys):
        k = _u64(keys)
        out = np.empty(k.size, dtype=np.uint64)
        fd = np.empty(k.size, dtype=np.uint8)
        if lib().or_part_find(self._h, _ptr(k), k.size, _ptr(out), (1 << 64) - 1, _ptr(fd)):
            raise MemoryError("partitioned find")
        return out, fd

    def erase(self, keys) -> np.ndarray:
        k = _u64(keys)
        er = np.empty(k.size, dtype=np.uint8)
        if lib().or_part_erase(self._h, _ptr(k), k.size, _ptr(er)):
            raise MemoryError("partitioned erase")
        return er


class OraclePool:
    """Fixed-capacity int32 stack (vector/deque back operations); fresh pools pop 0, 1, 2, ..."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity)
        self._h = lib().or_pool_new(self.capacity)
        if not self._h:
            raise MemoryError("oracle pool allocation failed")

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_pool_free(self._h)
            self._h = None

    def size(self) -> int:
        return int(lib().or_pool_size(self._h))

    def dump(self) -> np.ndarray:
        n = self.size()
        out = np.empty(n, dtype=np.int32)
        lib().or_pool_dump(self._h, _ptr(out), n)
        return out

    def pop(self, n: int):
        out = np.empty(int(n), dtype=np.int32)
        st = np.empty(int(n), dtype=np.uint8)
        lib().or_pool_pop(self._h, int(n), _ptr(out), _ptr(st))
        return out, st

    def push(self, values):
        v = np.ascontiguousarray(values, dtype=np.int32)
        st = np.empty(v.size, dtype=np.uint8)
        lib().or_pool_push(self._h, _ptr(v), v.size, _ptr(st))
        return st

    def pop_front(self, n: int):
        """pop_front n times (deque front operation, Section 4.3)."""
        out = np.empty(int(n), dtype=np.int32)
        st = np.empty(int(n), dtype=np.uint8)
        lib().or_pool_pop_front(self._h, int(n), _ptr(out), _ptr(st))
        return out, st

    def push_front(self, values):
        """push_front of each value in order: the last one ends up first."""
        v = np.ascontiguousarray(values, dtype=np.int32)
        st = np.empty(v.size, dtype=np.uint8)
        lib().or_pool_push_front(self._h, _ptr(v), v.size, _ptr(st))
        return st


def voxel_neighbour_keys(blocks, ndirs: int = 6) -> np.ndarray:
    """The 6 face (or all 26) neighbour keys of each packed voxel block, block by block in a fixed
    direction order; coordinates wrap in their 21-bit fields."""
    b = _u64(blocks)
    out = np.empty(b.size * ndirs, dtype=np.uint64)
    m = int(lib().or_voxel_neighbour_keys(_ptr(b), b.size, int(ndirs), _ptr(out)))
    if m < 0:
        raise ValueError("ndirs must be 6 or 26")
    return out


class OracleTable:
    """Sequential reference table: u64 keys, values of ``value_bits`` (0 = set, 32 or 64)."""

    def __init__(self, capacity: int, value_bits: int = 64, hash_kind: int = HASH_MIX64,
                 bucket_count: int | None = None):
        self.capacity = int(capacity)
        self.value_bits = int(value_bits)
        self.hash_kind = int(hash_kind)
        nb = int(bucket_count) if bucket_count else max(1, self.capacity)
        self.bucket_count = nb
        self._h = lib().or_table_new(self.capacity, self.hash_kind, nb)
        if not self._h:
            raise MemoryError("oracle table allocation failed")

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_table_free(self._h)
            self._h = None

    @property
    def sentinel(self) -> int:
        return (1 << 32) - 1 if self.value_bits == 32 else (1 << 64) - 1

    def _vals_in(self, vals, n):
        if self.value_bits == 0 or vals is None:
            return np.zeros(n, dtype=np.uint64)
        v = np.asarray(vals)
        if self.value_bits == 32:
            return np.ascontiguousarray(v.astype(np.int64).astype(np.uint64) & np.uint64(0xFFFFFFFF)
                                        if v.dtype.kind == "i" else v.astype(np.uint64))
        return _u64(v)

    def size(self) -> int:
        return int(lib().or_size(self._h))

    def error(self) -> int:
        return int(lib().or_error(self._h))

    def clear(self):
        lib().or_clear(self._h)

    def bucket_of(self, key: int) -> int:
        return int(lib().or_bucket_of(self._h, int(key)))

    def insert(self, keys, vals=None) -> np.ndarray:
        k = _u64(keys)
        v = self._vals_in(vals, k.size)
        st = np.empty(k.size, dtype=np.uint8)
        lib().or_insert(self._h, _ptr(k), _ptr(v), k.size, _ptr(st))
        return st

    def find(self, keys):
        """Returns (values, found); values are uint32/uint64 by width, the all-ones sentinel when absent."""
        k = _u64(keys)
        out = np.empty(k.size, dtype=np.uint64)
        fd = np.empty(k.size, dtype=np.uint8)
        lib().or_find(self._h, _ptr(k), k.size, _ptr(out), self.sentinel, _ptr(fd))
        if self.value_bits == 32:
            out = out.astype(np.uint32)
        return out, fd

    def erase(self, keys) -> np.ndarray:
        k = _u64(keys)
        er = np.empty(k.size, dtype=np.uint8)
        lib().or_erase(self._h, _ptr(k), k.size, _ptr(er))
        return er

    def insert_alloc(self, pool: OraclePool, keys):
        k = _u64(keys)
        out = np.empty(k.size, dtype=np.int32)
        st = np.empty(k.size, dtype=np.uint8)
        lib().or_insert_alloc(self._h, pool._h, _ptr(k), k.size, _ptr(out), _ptr(st))
        return out, st

    def erase_release(self, pool: OraclePool, keys) -> np.ndarray:
        k = _u64(keys)
        er = np.empty(k.size, dtype=np.uint8)
        lib().or_erase_release(self._h, pool._h, _ptr(k), k.size, _ptr(er))
        return er

    def dump(self):
        """Live (keys, values) sorted by key."""
        n = self.size()
        ks = np.empty(n, dtype=np.uint64)
        vs = np.empty(n, dtype=np.uint64)
        lib().or_dump(self._h, _ptr(ks), _ptr(vs), n)
        if self.value_bits == 32:
            vs = vs.astype(np.uint32)
        return ks, vs

    def select_key_range(self, lo: int, hi: int):
        """Live (keys, values) with lo <= key < hi, sorted by key (range selection, Section 3.6)."""
        return self._select(0, lo, hi, (0, 0, 0), (0, 0, 0))

    def select_voxel_box(self, lo3, hi3):
        """Live (keys, values) whose packed block coordinates lie in the box [lo3, hi3] (bounds
        included), sorted by key."""
        return self._select(1, 0, 0, lo3, hi3)

    def _select(self, kind, lo, hi, lo3, hi3):
        l3 = np.ascontiguousarray(lo3, dtype=np.int32)
        h3 = np.ascontiguousarray(hi3, dtype=np.int32)
        n = int(lib().or_select(self._h, kind, int(lo), int(hi), _ptr(l3), _ptr(h3), None, None, 0))
        ks = np.empty(n, dtype=np.uint64)
        vs = np.empty(n, dtype=np.uint64)
        lib().or_select(self._h, kind, int(lo), int(hi), _ptr(l3), _ptr(h3), _ptr(ks), _ptr(vs), n)
        if self.value_bits == 32:
            vs = vs.astype(np.uint32)
        return ks, vs

    def check(self, pool: OraclePool | None = None, values_from_pool: bool = False):
        """(violations, bitmask of failed invariants) -- see ``or_check`` in oracle.c."""
        w = C.c_int(0)
        bad = lib().or_check(self._h, pool._h if pool is not None else None, int(values_from_pool),
                             C.byref(w))
        return int(bad), int(w.value)

    def corrupt(self, kind: int, pool: OraclePool | None = None) -> bool:
        """TEST HOOK: break exactly one invariant (``or_corrupt`` in oracle.c lists the kinds) so a
        test can show that ``check`` reports it.  False when the state has no room for it."""
        return lib().or_corrupt(self._h, pool._h if pool is not None else None, int(kind)) == 0
