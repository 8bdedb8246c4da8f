"""Python binding of the FCIQMC C ABI (include/fciqmc.h).

Argument marshalling only: every step of an iteration runs in the HIP kernels
of ``libfqgpu.so``. PyTorch supplies the device workspace (a uint8 tensor) and
the stream. There is no CPU fallback: without the built library on a GPU
machine every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfqgpu.so")

FQ_OK, FQ_EINVAL, FQ_ECAPACITY, FQ_EOVERFLOW, FQ_EHIP, FQ_ESTATE, FQ_ENOREF = 0, -1, -2, -3, -4, -5, -6
HUBBARD, UEG, MOLECULAR = 1, 2, 3
EXGEN = {HUBBARD: 1, UEG: 2, MOLECULAR: 3}
SS_FP64, SS_SPLIT_BF16 = 0, 1
FCIQMC, DMQMC, IPDMQMC, CCMC = 0, 1, 2, 3

# every function the header declares
C_API = ["fq_workspace_bytes", "fq_init_system", "fq_init_system_static", "fq_step", "fq_estimators", "fq_estimator_history",
         "fq_export_walkers", "fq_import_walkers", "fq_shift_state", "fq_export_spawns", "fq_detspace", "fq_info",
         "fq_set_timing", "fq_stage_times", "fq_kernel_times", "fq_iteration_times", "fq_set_graph",
         "fq_set_sort_key_bits", "fq_set_launch", "fq_get_launch", "fq_set_tiles", "fq_get_tiles",
         "fq_reblock_create", "fq_reblock_add",
         "fq_reblock_level", "fq_reblock_optimal", "fq_reblock_ratio", "fq_reblock_destroy", "fq_last_error",
         "fq_destroy"]
LAUNCH_KERNELS = ["spawn", "merge", "sort", "reduce", "new_diag"]
# tile shapes (fq_set_tiles): spawning attempts, merge positions and sort keys per thread
TILE_KNOBS = ["spawn_items", "merge_items", "sort_items"]
TILE_VARIANTS = {"spawn_items": (2, 4, 8), "merge_items": (1, 2, 4), "sort_items": (8, 12, 16)}

KERNEL_SLOTS = ["begin", "spawn_partition", "spawn", "ccmc_clusters", "sort_hist"] + \
    [f"sort_pass{p}" for p in range(8)] + ["reduce", "fixup", "reduce2", "det_gather", "det_project", "det_check",
                                            "merge_partition", "merge", "new_diag", "ccmc_pairs", "end"]


class FqError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fciqmc error {code}: {msg}")
        self.code = code


class System(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_alpha", C.c_int32), ("n_beta", C.c_int32),
                ("n_sites", C.c_int32), ("periodic", C.c_int32), ("t", C.c_double), ("U", C.c_double),
                ("rs", C.c_double), ("ecut_n2", C.c_int32), ("n_orb", C.c_int32),
                ("h1", C.POINTER(C.c_double)), ("eri", C.POINTER(C.c_double))]


class Qmc(C.Structure):
    _fields_ = [("tau", C.c_double), ("rng_seed", C.c_uint64), ("replica_id", C.c_int32),
                ("init_pop", C.c_double), ("target_population", C.c_double),
                ("shift_period", C.c_int32), ("shift_damping", C.c_double), ("initial_shift", C.c_double),
                ("excit_gen", C.c_int32), ("p_single", C.c_double), ("initiator", C.c_int32),
                ("initiator_threshold", C.c_double), ("fixed_point_bits", C.c_int32),
                ("spawn_cutoff", C.c_double), ("tau_search", C.c_int32), ("method", C.c_int32),
                ("ccmc_truncation", C.c_int32)]


class SemiStoch(C.Structure):
    _fields_ = [("size", C.c_int32), ("start_iteration", C.c_int32), ("precision", C.c_int32),
                ("check_period", C.c_int32), ("shared", C.c_int32)]


class Estimators(C.Structure):
    _fields_ = [("iteration", C.c_int64), ("n_walkers_units", C.c_int64), ("n_occupied", C.c_int64),
                ("n_spawned", C.c_int64), ("ref_pop_units", C.c_int64), ("n_sign_flips", C.c_int64),
                ("n_rejected_units", C.c_int64), ("n_spawn_events", C.c_int64),
                ("death_sum", C.c_int64), ("spawn_sum", C.c_int64), ("rejected_sum", C.c_int64),
                ("vary_shift", C.c_int32), ("status", C.c_int32), ("shift", C.c_double),
                ("proj_numerator", C.c_double), ("proj_energy", C.c_double), ("e_ref", C.c_double),
                ("num_limbs", C.c_int64 * 4), ("ss_error", C.c_double), ("ss_error_bound", C.c_double),
                ("tau", C.c_double), ("spawn_ratio_max", C.c_double), ("pair_limbs", C.c_int64 * 4),
                ("n_cluster_spawns", C.c_int64)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f not in ("num_limbs", "pair_limbs")}
        d["num_limbs"] = list(self.num_limbs)
        d["pair_limbs"] = list(self.pair_limbs)
        return d


_lib = None


def load_library():
    """Loads the in-tree HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1811_11679_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    L.fq_workspace_bytes.argtypes = [C.POINTER(System), C.POINTER(Qmc), C.POINTER(SemiStoch), C.c_int32,
                                     C.c_int64, C.c_int64]
    L.fq_workspace_bytes.restype = C.c_size_t
    L.fq_init_system.argtypes = [C.POINTER(P), C.POINTER(System), C.POINTER(Qmc), C.POINTER(SemiStoch),
                                 C.c_int32, C.c_int64, C.c_int64, P, C.c_size_t, P]
    L.fq_init_system.restype = C.c_int32
    L.fq_init_system_static.argtypes = [C.POINTER(P), C.POINTER(System), C.POINTER(Qmc), C.POINTER(SemiStoch),
                                        C.c_int32, C.c_int64, C.c_int64, P]
    L.fq_init_system_static.restype = C.c_int32
    L.fq_step.argtypes = [P, C.c_int32]
    L.fq_step.restype = C.c_int32
    L.fq_estimators.argtypes = [P, C.c_int32, C.POINTER(Estimators)]
    L.fq_estimators.restype = C.c_int32
    L.fq_estimator_history.argtypes = [P, C.c_int32, C.POINTER(Estimators), C.c_int32, C.POINTER(C.c_int32)]
    L.fq_estimator_history.restype = C.c_int32
    L.fq_export_walkers.argtypes = [P, C.c_int32, P, P, C.c_int64, C.POINTER(C.c_int64)]
    L.fq_export_walkers.restype = C.c_int32
    L.fq_import_walkers.argtypes = [P, C.c_int32, P, P, C.c_int64, C.c_double, C.c_int64, C.c_int32,
                                    C.c_int64]
    L.fq_import_walkers.restype = C.c_int32
    L.fq_export_spawns.argtypes = [P, C.c_int32, P, P, P, C.c_int64, C.POINTER(C.c_int64)]
    L.fq_export_spawns.restype = C.c_int32
    L.fq_detspace.argtypes = [P, C.c_int32, P, P, C.c_int64, C.POINTER(C.c_int64)]
    L.fq_detspace.restype = C.c_int32
    L.fq_info.argtypes = [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double)]
    L.fq_info.restype = C.c_int32
    L.fq_set_timing.argtypes = [P, C.c_int32]
    L.fq_set_timing.restype = C.c_int32
    L.fq_stage_times.argtypes = [P, C.POINTER(C.c_double)]
    L.fq_stage_times.restype = C.c_int32
    L.fq_kernel_times.argtypes = [P, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int64)]
    L.fq_kernel_times.restype = C.c_int32
    L.fq_iteration_times.argtypes = [P, C.POINTER(C.c_double), C.c_int64, C.POINTER(C.c_int64)]
    L.fq_iteration_times.restype = C.c_int32
    L.fq_shift_state.argtypes = [P, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                 C.POINTER(C.c_int32)]
    L.fq_shift_state.restype = C.c_int32
    L.fq_set_graph.argtypes = [P, C.c_int32]
    L.fq_set_graph.restype = C.c_int32
    L.fq_set_sort_key_bits.argtypes = [P, C.c_int32]
    L.fq_set_sort_key_bits.restype = C.c_int32
    D = C.POINTER(C.c_double)
    L.fq_reblock_create.argtypes = [C.POINTER(P), C.c_int32, C.c_int32]
    L.fq_reblock_create.restype = C.c_int32
    L.fq_reblock_add.argtypes = [P, D]
    L.fq_reblock_add.restype = C.c_int32
    L.fq_reblock_level.argtypes = [P, C.c_int32, C.POINTER(C.c_int64), D, D]
    L.fq_reblock_level.restype = C.c_int32
    L.fq_reblock_optimal.argtypes = [P, C.c_int32, C.POINTER(C.c_int32)]
    L.fq_reblock_optimal.restype = C.c_int32
    L.fq_reblock_ratio.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, D, D]
    L.fq_reblock_ratio.restype = C.c_int32
    L.fq_reblock_destroy.argtypes = [P]
    L.fq_reblock_destroy.restype = None
    L.fq_set_launch.argtypes = [P, C.POINTER(C.c_int32), C.c_int32]
    L.fq_set_launch.restype = C.c_int32
    L.fq_get_launch.argtypes = [P, C.POINTER(C.c_int32), C.c_int32]
    L.fq_get_launch.restype = C.c_int32
    L.fq_set_tiles.argtypes = [P, C.POINTER(C.c_int32), C.c_int32]
    L.fq_set_tiles.restype = C.c_int32
    L.fq_get_tiles.argtypes = [P, C.POINTER(C.c_int32), C.c_int32]
    L.fq_get_tiles.restype = C.c_int32
    L.fq_last_error.argtypes = [P]
    L.fq_last_error.restype = C.c_char_p
    L.fq_destroy.argtypes = [P]
    _lib = L
    return L


def make_system(kind, **kw):
    s = System()
    s.kind = kind
    s.n_alpha = kw.get("n_alpha", 0)
    s.n_beta = kw.get("n_beta", 0)
    s.n_sites = kw.get("n_sites", 0)
    s.periodic = int(kw.get("periodic", 1))
    s.t = kw.get("t", 1.0)
    s.U = kw.get("U", 0.0)
    s.rs = kw.get("rs", 0.0)
    s.ecut_n2 = kw.get("ecut_n2", 0)
    keep = []
    if kind == MOLECULAR:
        h1 = np.ascontiguousarray(kw["h1"], np.float64)
        eri = np.ascontiguousarray(kw["eri"], np.float64)
        keep = [h1, eri]
        s.n_orb = h1.shape[0]
        s.h1 = h1.ctypes.data_as(C.POINTER(C.c_double))
        s.eri = eri.ctypes.data_as(C.POINTER(C.c_double))
    return s, keep


def make_qmc(**kw):
    d = dict(tau=0.01, rng_seed=7, replica_id=0, init_pop=500.0, target_population=1e4, shift_period=10,
             shift_damping=0.05, initial_shift=0.0, excit_gen=1, p_single=0.1, initiator=0,
             initiator_threshold=3.0, fixed_point_bits=0, spawn_cutoff=0.0, tau_search=0)
    d.update(kw)
    return Qmc(**d)


class Context:
    """One FCIQMC context on a HIP device: n_instances replicas of one system shape."""

    def __init__(self, systems, qmcs, semistoch=None, main_capacity=1 << 16, spawn_capacity=1 << 16,
                 device="cuda:0", stream=None, graph=False, static_workspace=False):
        import torch

        L = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device available")
        self.torch = torch
        self.R = len(systems)
        assert len(qmcs) == self.R
        sysarr = (System * self.R)()
        self._keep = []
        for i, (s, keep) in enumerate(systems):
            sysarr[i] = s
            self._keep += keep
        qarr = (Qmc * self.R)(*qmcs)
        ssarr = None
        if semistoch is not None:
            ssarr = (SemiStoch * self.R)(*([semistoch] * self.R))
        self._sys, self._q, self._ss = sysarr, qarr, ssarr
        nbytes = L.fq_workspace_bytes(sysarr, qarr, ssarr, self.R, main_capacity, spawn_capacity)
        if nbytes == 0:
            raise FqError(FQ_EINVAL, "invalid system description")
        self.device = torch.device(device)
        self.n_cu = torch.cuda.get_device_properties(self.device).multi_processor_count
        if stream is None and graph:
            stream = torch.cuda.Stream(self.device)  # default priority; graph capture needs a real stream
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = C.c_void_p()
        if static_workspace:
            # the library's static device array (fq_init_system_static): no workspace allocated here
            self.workspace = None
            with torch.cuda.device(self.device):
                st = L.fq_init_system_static(C.byref(self.ctx), sysarr, qarr, ssarr, self.R, main_capacity,
                                             spawn_capacity, C.c_void_p(self.stream.cuda_stream))
            if st != FQ_OK:
                raise FqError(st, "fq_init_system_static failed")
        else:
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            off = (-base) % 256
            st = L.fq_init_system(C.byref(self.ctx), sysarr, qarr, ssarr, self.R, main_capacity, spawn_capacity,
                                  C.c_void_p(base + off), nbytes, C.c_void_p(self.stream.cuda_stream))
            if st != FQ_OK:
                raise FqError(st, "fq_init_system failed")
        self.lib = L
        W, nso, e0 = C.c_int32(), C.c_int32(), C.c_double()
        L.fq_info(self.ctx, C.byref(W), C.byref(nso), C.byref(e0))
        self.W, self.n_so, self.e_ref = W.value, nso.value, e0.value
        self.main_capacity, self.spawn_capacity = main_capacity, spawn_capacity
        if graph:
            self._check(L.fq_set_graph(self.ctx, 1))

    def _check(self, st):
        if st != FQ_OK:
            raise FqError(st, self.lib.fq_last_error(self.ctx).decode())

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.fq_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        self._check(self.lib.fq_step(self.ctx, n))

    def estimators(self, instance=0):
        e = Estimators()
        self._check(self.lib.fq_estimators(self.ctx, instance, C.byref(e)))
        return e.as_dict()

    def history(self, instance=0, cap=1 << 16):
        arr = (Estimators * cap)()
        n = C.c_int32()
        self._check(self.lib.fq_estimator_history(self.ctx, instance, arr, cap, C.byref(n)))
        return [arr[i].as_dict() for i in range(n.value)]

    def export(self, instance=0):
        n = C.c_int64()
        st = self.lib.fq_export_walkers(self.ctx, instance, None, None, 0, C.byref(n))
        if st not in (FQ_OK, FQ_ECAPACITY):
            self._check(st)
        keys = np.zeros(max(n.value, 1) * self.W, np.uint64)
        pops = np.zeros(max(n.value, 1), np.int32)
        self._check(self.lib.fq_export_walkers(self.ctx, instance, keys.ctypes.data, pops.ctypes.data,
                                               n.value, C.byref(n)))
        return keys[: n.value * self.W].reshape(n.value, self.W), pops[: n.value]

    def import_walkers(self, keys, pops, instance=0, shift=0.0, iteration=0, vary=0, n_prev=0):
        keys = np.ascontiguousarray(keys, np.uint64).reshape(-1)
        pops = np.ascontiguousarray(pops, np.int32)
        self._check(self.lib.fq_import_walkers(self.ctx, instance, keys.ctypes.data, pops.ctypes.data,
                                               len(pops), shift, iteration, vary, n_prev))

    def shift_state(self, instance=0):
        """(shift, n_prev, vary): with export() and estimators(), what import_walkers needs"""
        sh, npv, va = C.c_double(), C.c_int64(), C.c_int32()
        self._check(self.lib.fq_shift_state(self.ctx, instance, C.byref(sh), C.byref(npv), C.byref(va)))
        return sh.value, npv.value, va.value

    def spawns(self, instance=0):
        n = C.c_int64()
        self.lib.fq_export_spawns(self.ctx, instance, None, None, None, 0, C.byref(n))
        keys = np.zeros(max(n.value, 1) * self.W, np.uint64)
        amps = np.zeros(max(n.value, 1), np.int32)
        init = np.zeros(max(n.value, 1), np.uint8)
        self._check(self.lib.fq_export_spawns(self.ctx, instance, keys.ctypes.data, amps.ctypes.data,
                                              init.ctypes.data, n.value, C.byref(n)))
        return keys[: n.value * self.W].reshape(n.value, self.W), amps[: n.value], init[: n.value]

    def detspace(self, instance=0):
        n = C.c_int64()
        st = self.lib.fq_detspace(self.ctx, instance, None, None, 0, C.byref(n))
        if st not in (FQ_OK, FQ_ECAPACITY):
            self._check(st)
        keys = np.zeros(max(n.value, 1) * self.W, np.uint64)
        y = np.zeros(max(n.value, 1), np.float64)
        self._check(self.lib.fq_detspace(self.ctx, instance, keys.ctypes.data, y.ctypes.data, n.value,
                                         C.byref(n)))
        return keys[: n.value * self.W].reshape(n.value, self.W), y[: n.value]

    def set_graph(self, on=True):
        self._check(self.lib.fq_set_graph(self.ctx, int(on)))

    def set_sort_key_bits(self, bits):
        """Only the top `bits` hash bits enter the sort keys (hash-collision tests)."""
        self._check(self.lib.fq_set_sort_key_bits(self.ctx, int(bits)))

    def set_launch(self, blocks):
        """blocks: {kernel name: blocks} for names in LAUNCH_KERNELS"""
        arr = (C.c_int32 * len(LAUNCH_KERNELS))(*[int(blocks.get(k, 0)) for k in LAUNCH_KERNELS])
        self._check(self.lib.fq_set_launch(self.ctx, arr, len(LAUNCH_KERNELS)))

    def get_launch(self):
        arr = (C.c_int32 * len(LAUNCH_KERNELS))()
        self._check(self.lib.fq_get_launch(self.ctx, arr, len(LAUNCH_KERNELS)))
        return dict(zip(LAUNCH_KERNELS, list(arr)))

    def set_tiles(self, tiles):
        """tiles: {name: value} for names in TILE_KNOBS (see fq_set_tiles)"""
        arr = (C.c_int32 * len(TILE_KNOBS))(*[int(tiles.get(k, 0)) for k in TILE_KNOBS])
        self._check(self.lib.fq_set_tiles(self.ctx, arr, len(TILE_KNOBS)))

    def get_tiles(self):
        arr = (C.c_int32 * len(TILE_KNOBS))()
        self._check(self.lib.fq_get_tiles(self.ctx, arr, len(TILE_KNOBS)))
        return dict(zip(TILE_KNOBS, list(arr)))

    def set_timing(self, on=True):
        self._check(self.lib.fq_set_timing(self.ctx, int(on)))

    def stage_times(self):
        arr = (C.c_double * 7)()
        self._check(self.lib.fq_stage_times(self.ctx, arr))
        names = ["scan", "spawn", "sort", "reduce", "merge", "detproj", "iteration"]
        return dict(zip(names, list(arr)))

    def iteration_times(self, cap=1 << 20):
        """device ms of each iteration of the last timed step call"""
        arr = (C.c_double * cap)()
        n = C.c_int64()
        self._check(self.lib.fq_iteration_times(self.ctx, arr, cap, C.byref(n)))
        return list(arr[: n.value])

    def kernel_times(self):
        """{slot name: summed ms}, and the number of timed iterations"""
        arr = (C.c_double * len(KERNEL_SLOTS))()
        ns, ni = C.c_int32(), C.c_int64()
        self._check(self.lib.fq_kernel_times(self.ctx, arr, len(KERNEL_SLOTS), C.byref(ns), C.byref(ni)))
        return dict(zip(KERNEL_SLOTS, list(arr))), ni.value
