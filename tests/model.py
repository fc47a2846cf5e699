"""Brute-force dictionary model of the hash-map semantics, used only to pin the
oracle on tiny inputs.  It is written independently of oracle/ (a Python dict
and a Python list for the index heap) and is deliberately naive."""


class DictModel:
    def __init__(self, capacity, n_values=0):
        self.c = capacity
        self.table = {}                     # key tuple -> buffer index
        self.heap = list(range(capacity))   # index heap h
        self.top = 0                        # heap top t
        self.values = {}                    # buffer index -> tuple of value rows
        self.n_values = n_values

    def _grow_to(self, new_c):
        self.heap.extend(range(self.c, new_c))
        self.c = new_c

    def insert(self, keys, values=None, autogrow=False, activate=False):
        new = []
        for k in keys:
            if k not in self.table and k not in new:
                new.append(k)
        if len(new) > self.c - self.top:
            if not autogrow:
                return 2, [-1] * len(keys), [0] * len(keys)
            c = max(self.c, 1)
            while c - self.top < len(new):
                c *= 2
            self._grow_to(c)
        idx, mask = [], []
        for p, k in enumerate(keys):
            if k in self.table:
                idx.append(-1)
                mask.append(0)
                continue
            i = self.heap[self.top]
            self.top += 1
            self.table[k] = i
            if not activate:
                self.values[i] = tuple(v[p] for v in values) if values else ()
            idx.append(i)
            mask.append(1)
        return 0, idx, mask

    def find(self, keys):
        idx = [self.table.get(k, -1) for k in keys]
        return idx, [int(i >= 0) for i in idx]

    def erase(self, keys):
        mask = []
        for k in keys:
            if k in self.table:
                i = self.table.pop(k)
                self.top -= 1
                self.heap[self.top] = i
                mask.append(1)
            else:
                mask.append(0)
        return mask

    def active(self):
        return sorted(self.table.values())
