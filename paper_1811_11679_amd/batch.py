"""Many independent FCIQMC instances advanced together on one GPU.

Instances whose determinants need the same number of 64-bit key words share
one library context: their walker lists live in one sorted array with the
replica id as the most significant sort digit, so every kernel of an
iteration covers all of them in one launch. Contexts of different key widths
run side by side on streams of their own (default priority), each replaying a
captured graph per block of shift-update iterations, driven from one host
thread per context (the library releases the interpreter lock while it waits).

Grouping by key width is host orchestration only; every step of the
iteration runs in the library's kernels.
"""
from __future__ import annotations

import threading

from . import fciqmc as F


def n_plane_waves(ecut_n2: int) -> int:
    """Number of integer vectors n with |n|^2 <= ecut_n2 (the basis of the
    simple-cubic electron gas, Sec. 4.3)."""
    m = int(ecut_n2 ** 0.5) + 1
    return sum(1 for x in range(-m, m + 1) for y in range(-m, m + 1) for z in range(-m, m + 1)
               if x * x + y * y + z * z <= ecut_n2)


def spin_orbitals(system: dict) -> int:
    kind = system["kind"]
    if kind == "hubbard":
        return 2 * system["n_sites"]
    if kind == "ueg":
        return 2 * n_plane_waves(system["ecut_n2"])
    return 2 * system["n_orb"]


def key_words(system: dict) -> int:
    """64-bit words per determinant key as the library stores it (1, 2, 4 or 8)."""
    w = (spin_orbitals(system) + 63) // 64
    for c in (1, 2, 4, 8):
        if w <= c:
            return c
    raise ValueError("more than 512 spin-orbitals")


KIND = {"hubbard": F.HUBBARD, "ueg": F.UEG, "molecular": F.MOLECULAR}


class Batch:
    """Independent instances grouped into one context per (kind, key width).

    instances: list of (system dict, qmc dict); qmc dicts carry replica_id.
    capacity(group) -> (main_capacity, spawn_capacity) for a list of instance
    indices. Instance i of the batch is reached as (group, slot) = where[i].
    """

    def __init__(self, instances, capacity, device="cuda:0", graph=True, ints=None):
        groups = {}
        for i, (sysd, q) in enumerate(instances):
            groups.setdefault((sysd["kind"], key_words(sysd)), []).append(i)
        self.groups = [groups[k] for k in sorted(groups)]
        self.where = {}
        self.contexts = []
        for g, members in enumerate(self.groups):
            systems, qmcs = [], []
            for slot, i in enumerate(members):
                sysd, q = instances[i]
                kw = {x: v for x, v in sysd.items() if x != "kind"}
                if sysd["kind"] == "molecular":
                    kw["h1"], kw["eri"] = ints
                systems.append(F.make_system(KIND[sysd["kind"]], **kw))
                qq = dict(q)
                qq["excit_gen"] = KIND[sysd["kind"]]
                qmcs.append(F.make_qmc(**qq))
                self.where[i] = (g, slot)
            mc, sc = capacity(members)
            self.contexts.append(F.Context(systems, qmcs, main_capacity=mc, spawn_capacity=sc, device=device,
                                           graph=graph))

    def _each(self, fn):
        errors = [None] * len(self.contexts)

        def run(k):
            try:
                fn(self.contexts[k])
            except BaseException as e:  # re-raised on the calling thread
                errors[k] = e

        threads = [threading.Thread(target=run, args=(k,)) for k in range(len(self.contexts))]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        for e in errors:
            if e is not None:
                raise e

    def step(self, n=1):
        """Advance every instance by n iterations (all contexts concurrently)."""
        self._each(lambda c: c.step(n))

    def synchronize(self):
        for c in self.contexts:
            c.stream.synchronize()

    def estimators(self, i):
        g, slot = self.where[i]
        return self.contexts[g].estimators(slot)

    def history(self, i):
        g, slot = self.where[i]
        return self.contexts[g].history(slot)

    def export(self, i):
        g, slot = self.where[i]
        return self.contexts[g].export(slot)

    def shift_state(self, i):
        g, slot = self.where[i]
        return self.contexts[g].shift_state(slot)

    def close(self):
        for c in self.contexts:
            c.close()
        self.contexts = []
