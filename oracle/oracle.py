"""ctypes binding of the FCIQMC oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this module. The product path (``paper_1811_11679_amd``) never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fq_oracle.c")
LIB = os.path.join(HERE, "libfq_oracle.so")

HUBBARD, UEG, MOLECULAR = 1, 2, 3
EXGEN_HUB, EXGEN_UEG, EXGEN_HEATBATH = 1, 2, 3
FCIQMC, DMQMC, IPDMQMC, CCMC = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the oracle with gcc, FP contraction off (a plain C build)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "fq_oracle.h"))):
        cmd = ["gcc", "-std=gnu11", "-O2", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class Qmc(C.Structure):
    _fields_ = [("tau", C.c_double), ("seed", C.c_uint64), ("replica_id", C.c_int32),
                ("init_pop", C.c_double), ("target_population", C.c_double),
                ("shift_period", C.c_int32), ("shift_damping", C.c_double),
                ("initial_shift", C.c_double), ("excit_gen", C.c_int32),
                ("p_single", C.c_double), ("initiator", C.c_int32),
                ("initiator_threshold", C.c_double), ("fixed_point_bits", C.c_int32),
                ("spawn_cutoff", C.c_double), ("ss_size", C.c_int32),
                ("ss_start_iteration", C.c_int32), ("ss_shared", C.c_int32), ("tau_search", C.c_int32),
                ("method", C.c_int32), ("ccmc_truncation", C.c_int32)]


class Estimators(C.Structure):
    _fields_ = [("iteration", C.c_int64), ("n_walkers_units", C.c_int64),
                ("n_occupied", C.c_int64), ("n_spawned", C.c_int64),
                ("ref_pop_units", C.c_int64), ("n_sign_flips", C.c_int64),
                ("n_rejected_units", C.c_int64), ("n_spawn_events", C.c_int64),
                ("death_sum", C.c_int64), ("spawn_sum", C.c_int64), ("rejected_sum", C.c_int64),
                ("vary_shift", C.c_int32), ("status", C.c_int32),
                ("shift", C.c_double), ("proj_numerator", C.c_double),
                ("proj_energy", C.c_double), ("e_ref", C.c_double),
                ("num_limbs", C.c_int64 * 4), ("pair_limbs", C.c_int64 * 4), ("tau", C.c_double),
                ("spawn_ratio_max", C.c_double), ("n_cluster_spawns", C.c_int64)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f not in ("num_limbs", "pair_limbs")}
        d["num_limbs"] = list(self.num_limbs)
        d["pair_limbs"] = list(self.pair_limbs)
        return d


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        P = C.c_void_p
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C")
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C")
        L.or_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.or_hash64.argtypes = [u64p, C.c_int]
        L.or_hash64.restype = C.c_uint64
        L.or_hubbard_new.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int]
        L.or_hubbard_new.restype = P
        L.or_ueg_new.argtypes = [C.c_double, C.c_int, C.c_int, C.c_int]
        L.or_ueg_new.restype = P
        L.or_molecular_new.argtypes = [C.c_int, f64p, f64p, C.c_int, C.c_int]
        L.or_molecular_new.restype = P
        L.or_sys_free.argtypes = [P]
        L.or_sys_info.argtypes = [P, i32p, f64p]
        L.or_sys_reference.argtypes = [P, u64p]
        L.or_ueg_orbitals.argtypes = [P, i32p]
        L.or_heatbath_size.argtypes = [P]
        L.or_heatbath_size.restype = C.c_int64
        L.or_hij.argtypes = [P, u64p, u64p]
        L.or_hij.restype = C.c_double
        L.or_diag.argtypes = [P, u64p]
        L.or_diag.restype = C.c_double
        L.or_exgen.argtypes = [P, C.c_int, C.c_double, u64p, u32p, u64p,
                               C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.or_exgen.restype = C.c_int
        L.or_run_new.argtypes = [P, C.POINTER(Qmc)]
        L.or_run_new.restype = P
        L.or_run_free.argtypes = [P]
        L.or_run_step.argtypes = [P, C.c_int]
        L.or_run_step.restype = C.c_int
        L.or_runs_select_shared.argtypes = [C.POINTER(P), C.c_int]
        L.or_runs_select_shared.restype = C.c_int
        L.or_run_estimators.argtypes = [P, C.POINTER(Estimators)]
        L.or_run_size.argtypes = [P]
        L.or_run_size.restype = C.c_int64
        L.or_run_export.argtypes = [P, u64p, i32p]
        L.or_run_import.argtypes = [P, u64p, i32p, C.c_int64, C.c_double, C.c_int64,
                                    C.c_int32, C.c_int64]
        L.or_run_import.restype = C.c_int
        L.or_run_n_spawns.argtypes = [P]
        L.or_run_n_spawns.restype = C.c_int64
        L.or_run_spawns.argtypes = [P, u64p, i32p, u8p]
        L.or_run_detspace.argtypes = [P, C.c_void_p]
        L.or_run_detspace.restype = C.c_int64
        L.or_run_last_projection.argtypes = [P, f64p]
        L.or_cluster_collapse.argtypes = [P, u64p, C.c_int, u64p]
        L.or_cluster_collapse.restype = C.c_int
        _lib = L
    return _lib


def philox(ctr, key):
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def hash64(words):
    w = np.ascontiguousarray(words, dtype=np.uint64)
    return int(lib().or_hash64(w, len(w)))


class System:
    """An oracle system (Hubbard ring, uniform electron gas, molecular)."""

    def __init__(self, ptr, keepalive=()):
        if not ptr:
            raise ValueError("invalid system parameters")
        self.ptr = ptr
        self._keep = keepalive
        iout = np.zeros(7, np.int32)
        dout = np.zeros(4, np.float64)
        lib().or_sys_info(ptr, iout, dout)
        (self.kind, self.n_spatial, self.n_so, self.W, self.nel,
         self.n_alpha, self.n_beta) = (int(x) for x in iout)
        self.H00, self.L, self.k2, self.vc = (float(x) for x in dout)
        self.ref = np.zeros(self.W, np.uint64)
        lib().or_sys_reference(ptr, self.ref)

    @classmethod
    def hubbard(cls, n_sites=8, periodic=True, t=1.0, U=4.0, n_alpha=4, n_beta=4):
        return cls(lib().or_hubbard_new(n_sites, int(periodic), t, U, n_alpha, n_beta))

    @classmethod
    def ueg(cls, rs=1.0, ecut=5, n_alpha=7, n_beta=7):
        return cls(lib().or_ueg_new(rs, ecut, n_alpha, n_beta))

    @classmethod
    def molecular(cls, h1, eri, n_alpha, n_beta):
        h1 = np.ascontiguousarray(h1, np.float64)
        eri = np.ascontiguousarray(eri, np.float64)
        return cls(lib().or_molecular_new(h1.shape[0], h1, eri, n_alpha, n_beta), (h1, eri))

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.or_sys_free(self.ptr)
            self.ptr = None

    def orbitals(self):
        nv = np.zeros(3 * self.n_spatial, np.int32)
        lib().or_ueg_orbitals(self.ptr, nv)
        return nv.reshape(-1, 3)

    def heatbath_size(self):
        return int(lib().or_heatbath_size(self.ptr))

    def hij(self, bra, ket):
        return float(lib().or_hij(self.ptr, np.asarray(bra, np.uint64), np.asarray(ket, np.uint64)))

    def diag(self, key):
        return float(lib().or_diag(self.ptr, np.asarray(key, np.uint64)))

    def cluster_collapse(self, excitors):
        """a_{e_1} ... a_{e_n} D_0 = sign D (CCMC excitors, a_e D_0 = +D_e):
        (sign, D), sign 0 when the product vanishes"""
        ex = np.ascontiguousarray(np.asarray(excitors, np.uint64).reshape(-1))
        out = np.zeros(self.W, np.uint64)
        sg = int(lib().or_cluster_collapse(self.ptr, ex, len(ex) // self.W, out))
        return sg, out

    def exgen(self, exgen, key, words, p_single=0.1):
        child = np.zeros(self.W, np.uint64)
        pg, h = C.c_double(), C.c_double()
        w = np.zeros(8, np.uint32)
        w[:len(words)] = words
        ok = lib().or_exgen(self.ptr, exgen, p_single, np.asarray(key, np.uint64), w, child,
                            C.byref(pg), C.byref(h))
        if not ok:
            return None
        return child, pg.value, h.value


def make_qmc(**kw) -> Qmc:
    d = dict(tau=0.01, seed=7, replica_id=0, init_pop=500.0, target_population=1e4,
             shift_period=10, shift_damping=0.05, initial_shift=0.0, excit_gen=EXGEN_HUB,
             p_single=0.1, initiator=0, initiator_threshold=3.0, fixed_point_bits=0,
             spawn_cutoff=0.0, ss_size=0, ss_start_iteration=0, ss_shared=0, tau_search=0, method=0,
             ccmc_truncation=0)
    d.update(kw)
    return Qmc(**d)


class Run:
    """One oracle FCIQMC run."""

    def __init__(self, system: System, qmc: Qmc):
        self.sys = system
        self.qmc = qmc
        self.ptr = lib().or_run_new(system.ptr, C.byref(qmc))
        if not self.ptr:
            raise ValueError("invalid qmc parameters")

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.or_run_free(self.ptr)
            self.ptr = None

    def step(self, n=1):
        st = lib().or_run_step(self.ptr, n)
        if st:
            raise RuntimeError(f"oracle step failed with status {st}")

    def estimators(self):
        e = Estimators()
        lib().or_run_estimators(self.ptr, C.byref(e))
        return e.as_dict()

    @property
    def W(self):
        """key words: the system's, doubled for the density-matrix methods"""
        return self.sys.W * (2 if self.qmc.method in (DMQMC, IPDMQMC) else 1)

    def export(self):
        n = int(lib().or_run_size(self.ptr))
        keys = np.zeros(max(n, 1) * self.W, np.uint64)
        pops = np.zeros(max(n, 1), np.int32)
        lib().or_run_export(self.ptr, keys, pops)
        return keys[: n * self.W].reshape(n, self.W), pops[:n]

    def import_walkers(self, keys, pops, shift=0.0, iteration=0, vary=0, n_prev=0):
        keys = np.ascontiguousarray(keys, np.uint64).reshape(-1)
        pops = np.ascontiguousarray(pops, np.int32)
        st = lib().or_run_import(self.ptr, keys, pops, len(pops), shift, iteration, vary, n_prev)
        if st:
            raise ValueError("import failed")

    def spawns(self):
        n = int(lib().or_run_n_spawns(self.ptr))
        keys = np.zeros(max(n, 1) * self.W, np.uint64)
        amps = np.zeros(max(n, 1), np.int32)
        init = np.zeros(max(n, 1), np.uint8)
        lib().or_run_spawns(self.ptr, keys, amps, init)
        return keys[: n * self.W].reshape(n, self.W), amps[:n], init[:n]

    def detspace(self):
        n = int(lib().or_run_detspace(self.ptr, None))
        keys = np.zeros(max(n, 1) * self.sys.W, np.uint64)
        lib().or_run_detspace(self.ptr, keys.ctypes.data)
        return keys[: n * self.sys.W].reshape(n, self.sys.W)

    def last_projection(self):
        n = int(lib().or_run_detspace(self.ptr, None))
        y = np.zeros(max(n, 1), np.float64)
        lib().or_run_last_projection(self.ptr, y)
        return y[:n]


def select_shared(runs):
    """Choose one deterministic space for runs of one system (qmc.ss_shared = 1)
    from their current lists."""
    arr = (C.c_void_p * len(runs))(*[r.ptr for r in runs])
    st = lib().or_runs_select_shared(arr, len(runs))
    if st:
        raise RuntimeError(f"shared deterministic space selection failed with status {st}")


def step_shared(runs, n):
    """Advance runs that share one deterministic space (qmc.ss_shared = 1) by n
    iterations: each iteration steps every run, and at the end of iteration
    ss_start_iteration D is chosen jointly over the runs."""
    for _ in range(n):
        for r in runs:
            r.step(1)
        q = runs[0].qmc
        if q.ss_size > 0 and runs[0].estimators()["iteration"] == q.ss_start_iteration:
            select_shared(runs)
