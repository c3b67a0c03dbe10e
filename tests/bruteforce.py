"""Brute-force model of the batch container operations for tiny inputs.

A list of [key, value] pairs scanned linearly and a Python list used as a stack: the most direct
reading of the sequential semantics (Section 4: fixed capacity, FULL as the only failure;
Section 4.1: unique keys, insert leaves a present key unmodified, find/erase; Sections 4.2-4.3:
push_back / pop_back at the end of the stack).  It pins the oracle; it shares no code with it.
"""

PRESENT, INSERTED, FULL = 0, 1, 2


class BrutePool:
    def __init__(self, capacity):
        self.capacity = capacity
        self.stack = list(range(capacity - 1, -1, -1))

    def pop(self, n):
        out, st = [], []
        for _ in range(n):
            if self.stack:
                out.append(self.stack.pop())
                st.append(1)
            else:
                out.append(-1)
                st.append(2)
        return out, st

    def push(self, values):
        st = []
        for v in values:
            if len(self.stack) == self.capacity:
                st.append(2)
            else:
                self.stack.append(int(v))
                st.append(1)
        return st


class BruteTable:
    def __init__(self, capacity, value_bits=64):
        self.capacity = capacity
        self.value_bits = value_bits
        self.pairs = []

    @property
    def sentinel(self):
        return (1 << 32) - 1 if self.value_bits == 32 else (1 << 64) - 1

    def _where(self, key):
        for j, (k, _) in enumerate(self.pairs):
            if k == key:
                return j
        return -1

    def insert(self, keys, vals):
        st = []
        for k, v in zip(keys, vals):
            if self._where(k) >= 0:
                st.append(PRESENT)
            elif len(self.pairs) == self.capacity:
                st.append(FULL)
            else:
                self.pairs.append([k, v])
                st.append(INSERTED)
        return st

    def find(self, keys):
        out, fd = [], []
        for k in keys:
            j = self._where(k)
            out.append(self.pairs[j][1] if j >= 0 else self.sentinel)
            fd.append(1 if j >= 0 else 0)
        return out, fd

    def erase(self, keys):
        er = []
        for k in keys:
            j = self._where(k)
            if j >= 0:
                del self.pairs[j]
            er.append(1 if j >= 0 else 0)
        return er

    def insert_alloc(self, pool, keys):
        out, st = [], []
        for k in keys:
            j = self._where(k)
            if j >= 0:
                out.append(self.pairs[j][1])
                st.append(PRESENT)
            elif len(self.pairs) == self.capacity or not pool.stack:
                out.append(-1)
                st.append(FULL)
            else:
                v = pool.stack.pop()
                self.pairs.append([k, v])
                out.append(v)
                st.append(INSERTED)
        return out, st

    def erase_release(self, pool, keys):
        er = []
        for k in keys:
            j = self._where(k)
            if j >= 0:
                v = self.pairs[j][1]
                del self.pairs[j]
                if len(pool.stack) < pool.capacity:
                    pool.stack.append(v)
            er.append(1 if j >= 0 else 0)
        return er

    def dump(self):
        return sorted((k, v) for k, v in self.pairs)
