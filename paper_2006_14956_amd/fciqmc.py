"""Thin ctypes binding of libfciqmc.so with the C entry points' names.

Argument marshalling only: every step of the FCIQMC path runs in the HIP
library.  Importing this module does not load the library; the first call
does, and it raises if the library has not been built -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libfciqmc.so")

OK, EINVAL, ENOMEM, EOVERFLOW, EDEVICE, ESTATE = 0, -1, -2, -3, -4, -5
MODE_INTEGER, MODE_REAL = 0, 1
GEN_UNIFORM, GEN_LATTICE, GEN_PCHB, GEN_CS, GEN_PE = 0, 1, 2, 3, 4


class FciqmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fciqmc error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("tau", C.c_double), ("walker_target", C.c_double), ("n_initial", C.c_double),
                ("initiator_na", C.c_double), ("mode", C.c_int), ("c_min", C.c_double),
                ("excitgen", C.c_int), ("p_single", C.c_double), ("p_opp", C.c_double),
                ("seed", C.c_uint64), ("replica_id", C.c_uint64), ("shift_damping", C.c_double),
                ("shift_restore", C.c_double),
                ("shift_interval", C.c_int), ("ref_alpha", C.c_uint64), ("ref_beta", C.c_uint64),
                ("max_dets", C.c_int64), ("max_spawns", C.c_int64),
                ("hbm_budget_bytes", C.c_int64), ("buckets_log2", C.c_int), ("det_words", C.c_int),
                ("conv_tol", C.c_double), ("equil_steps", C.c_int), ("adaptive_shift", C.c_int),
                ("ref_rechoose", C.c_int)]


class StepStats(C.Structure):
    _fields_ = [("iter", C.c_int64), ("nw", C.c_double), ("nref", C.c_double),
                ("enum_", C.c_double), ("shift", C.c_double), ("e_proj", C.c_double),
                ("ndets", C.c_int64), ("attempts", C.c_int64), ("spawns", C.c_int64),
                ("vary_shift", C.c_int), ("retries", C.c_int)]


class EnergyReport(C.Structure):
    _fields_ = [("e_proj", C.c_double), ("e_proj_err", C.c_double), ("shift", C.c_double),
                ("shift_err", C.c_double), ("e_ref", C.c_double), ("n_samples", C.c_int64),
                ("first_step", C.c_int64), ("steps_done", C.c_int64), ("converged", C.c_int)]


class Checkpoint(C.Structure):
    _fields_ = [("iter", C.c_int64), ("shift", C.c_double), ("vary_shift", C.c_int),
                ("last_update_iter", C.c_int64), ("last_update_nw", C.c_double)]


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3


class RequestInfo(C.Structure):
    _fields_ = [("state", C.c_int), ("error", C.c_int), ("converged", C.c_int),
                ("steps", C.c_int64), ("attempts", C.c_int64), ("reserved_bytes", C.c_int64),
                ("t_arrival", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("energy", EnergyReport)]


class TuneReport(C.Structure):
    _fields_ = [("persistent", C.c_int), ("dets_per_bucket", C.c_int), ("grid_spawn", C.c_int), ("grid_annihilate", C.c_int),
                ("trials", C.c_int), ("steps", C.c_int64), ("rate_initial", C.c_double),
                ("rate_best", C.c_double)]


EXPORTS = ["fciqmc_params_default", "fciqmc_load_integrals", "fciqmc_init", "fciqmc_step",
           "fciqmc_energy", "fciqmc_get_walkers", "fciqmc_set_walkers", "fciqmc_get_checkpoint",
           "fciqmc_get_reference",
           "fciqmc_set_checkpoint", "fciqmc_matrix_elements", "fciqmc_matrix_elements_noalloc",
           "fciqmc_pchb_row",
           "fciqmc_run_device_bytes",
           "fciqmc_profile", "fciqmc_batch_create", "fciqmc_batch_add", "fciqmc_batch_remove",
           "fciqmc_batch_size", "fciqmc_batch_step", "fciqmc_batch_tune", "fciqmc_batch_profile",
           "fciqmc_batch_set_persistent",
           "fciqmc_batch_free", "fciqmc_estimate_bytes", "fciqmc_server_create",
           "fciqmc_server_submit", "fciqmc_server_poll", "fciqmc_server_info",
           "fciqmc_server_clock", "fciqmc_server_free", "fciqmc_set_core", "fciqmc_get_core", "fciqmc_get_core_row",
           "fciqmc_pair_create", "fciqmc_pair_step", "fciqmc_pair_pt2", "fciqmc_pair_free",
           "fciqmc_pair_rdm_enable", "fciqmc_pair_rdm",
           "fciqmc_free_run", "fciqmc_free_system", "fciqmc_last_error"]

_lib = None


def lib():
    """Load libfciqmc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FciqmcError(ESTATE, f"{LIB_PATH} is missing: build it with "
                                      "`python paper_2006_14956_amd/build.py`")
        # torch ships its own HIP runtime under the same soname as ROCm's; load
        # it first so the process holds one runtime and torch streams are valid
        # handles inside the library
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp, i64, u64, dbl = C.c_void_p, C.c_int64, C.c_uint64, C.c_double
        pu64, pdbl = C.POINTER(u64), C.POINTER(dbl)
        L.fciqmc_params_default.argtypes = [C.POINTER(Params)]
        L.fciqmc_params_default.restype = None
        L.fciqmc_load_integrals.argtypes = [C.c_int, C.c_int, C.c_int, dbl, pdbl, pdbl, i64,
                                            C.POINTER(vp)]
        L.fciqmc_init.argtypes = [vp, C.POINTER(Params), vp, C.POINTER(vp)]
        L.fciqmc_step.argtypes = [vp, C.c_int, C.POINTER(StepStats)]
        L.fciqmc_energy.argtypes = [vp, C.POINTER(EnergyReport)]
        L.fciqmc_get_walkers.argtypes = [vp, pu64, pdbl, i64, C.POINTER(i64)]
        L.fciqmc_set_walkers.argtypes = [vp, pu64, pdbl, i64]
        L.fciqmc_set_core.argtypes = [vp, i64, C.POINTER(i64)]
        L.fciqmc_get_core.argtypes = [vp, pu64, i64, C.POINTER(i64), C.POINTER(i64)]
        L.fciqmc_get_core_row.argtypes = [vp, i64, C.POINTER(C.c_int32), C.POINTER(C.c_double), i64,
                                          C.POINTER(i64)]
        L.fciqmc_get_checkpoint.argtypes = [vp, C.POINTER(Checkpoint)]
        L.fciqmc_get_reference.argtypes = [vp, C.POINTER(u64), C.POINTER(u64), pdbl]
        L.fciqmc_set_checkpoint.argtypes = [vp, C.POINTER(Checkpoint)]
        L.fciqmc_matrix_elements.argtypes = [vp, pu64, pu64, i64, pdbl]
        L.fciqmc_matrix_elements_noalloc.argtypes = [vp, pu64, pu64, i64, pdbl]
        L.fciqmc_pchb_row.argtypes = [vp, C.c_int, i64, pdbl, C.POINTER(C.c_int32), pdbl, pdbl]
        L.fciqmc_run_device_bytes.argtypes = [vp]
        L.fciqmc_run_device_bytes.restype = i64
        L.fciqmc_profile.argtypes = [vp, C.c_int, pdbl, C.POINTER(i64), C.POINTER(i64)]
        L.fciqmc_batch_create.argtypes = [vp, C.POINTER(vp)]
        L.fciqmc_batch_add.argtypes = [vp, vp]
        L.fciqmc_batch_remove.argtypes = [vp, vp]
        L.fciqmc_batch_size.argtypes = [vp]
        L.fciqmc_batch_step.argtypes = [vp, C.c_int, C.POINTER(StepStats)]
        L.fciqmc_batch_tune.argtypes = [vp, C.c_int, C.POINTER(TuneReport)]
        L.fciqmc_batch_profile.argtypes = [vp, C.c_int, pdbl, C.POINTER(i64)]
        L.fciqmc_batch_set_persistent.argtypes = [vp, C.c_int]
        L.fciqmc_batch_free.argtypes = [vp]
        L.fciqmc_batch_free.restype = None
        L.fciqmc_estimate_bytes.argtypes = [vp, C.POINTER(Params)]
        L.fciqmc_estimate_bytes.restype = i64
        L.fciqmc_server_create.argtypes = [i64, C.c_int, vp, C.POINTER(vp)]
        L.fciqmc_server_submit.argtypes = [vp, vp, C.POINTER(Params), C.c_int, i64, dbl,
                                           C.POINTER(i64)]
        L.fciqmc_server_poll.argtypes = [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.fciqmc_server_info.argtypes = [vp, i64, C.POINTER(RequestInfo)]
        L.fciqmc_server_clock.argtypes = [vp]
        L.fciqmc_server_clock.restype = dbl
        L.fciqmc_server_free.argtypes = [vp]
        L.fciqmc_pair_create.argtypes = [vp, vp, C.POINTER(vp)]
        L.fciqmc_pair_step.argtypes = [vp, C.c_int, C.POINTER(StepStats), C.POINTER(StepStats), pdbl]
        L.fciqmc_pair_pt2.argtypes = [vp, i64, pdbl, pdbl, C.POINTER(i64)]
        L.fciqmc_pair_free.argtypes = [vp]
        L.fciqmc_pair_rdm_enable.argtypes = [vp, C.c_int]
        L.fciqmc_pair_rdm.argtypes = [vp, pdbl, i64, C.POINTER(i64), pdbl, pdbl, C.POINTER(i64)]
        L.fciqmc_pair_free.restype = None
        L.fciqmc_server_free.restype = None
        L.fciqmc_free_run.argtypes = [vp]
        L.fciqmc_free_run.restype = None
        L.fciqmc_free_system.argtypes = [vp]
        L.fciqmc_free_system.restype = None
        L.fciqmc_last_error.argtypes = []
        L.fciqmc_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def fciqmc_last_error() -> str:
    return lib().fciqmc_last_error().decode()


def _check(rc):
    if rc != 0:
        raise FciqmcError(rc, fciqmc_last_error())


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def fciqmc_params_default(**overrides) -> Params:
    p = Params()
    lib().fciqmc_params_default(C.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


class System:
    def __init__(self, handle):
        self.handle = handle

    def free(self):
        if self.handle:
            lib().fciqmc_free_system(self.handle)
            self.handle = None


class Run:
    def __init__(self, handle, system):
        self.handle = handle
        self.system = system  # keep the system alive
        self.batch = None

    def free(self):
        if self.handle:
            lib().fciqmc_free_run(self.handle)
            if self.batch is not None:
                self.batch.members.remove(self)
                self.batch = None
            self.handle = None


class Batch:
    def __init__(self, handle):
        self.handle = handle
        self.members = []  # Run objects, in order of addition

    def free(self):
        if self.handle:
            lib().fciqmc_batch_free(self.handle)
            for r in self.members:
                r.batch = None
            self.members = []
            self.handle = None


def fciqmc_load_integrals(n_orb, n_alpha, n_beta, e_core, h1, eri) -> System:
    h = np.ascontiguousarray(h1, dtype=np.float64)
    e = np.ascontiguousarray(eri, dtype=np.float64)
    out = C.c_void_p()
    _check(lib().fciqmc_load_integrals(int(n_orb), int(n_alpha), int(n_beta), float(e_core),
                                       _p(h, C.c_double), _p(e, C.c_double), len(e),
                                       C.byref(out)))
    return System(out.value)


def _stream_ptr(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def fciqmc_init(system: System, params: Params, stream=None) -> Run:
    out = C.c_void_p()
    _check(lib().fciqmc_init(system.handle, C.byref(params), _stream_ptr(stream), C.byref(out)))
    return Run(out.value, system)


STATS_DTYPE = np.dtype([(n, np.int64 if t in (C.c_int64,) else (np.int32 if t is C.c_int else np.float64))
                        for n, t in StepStats._fields_])


assert STATS_DTYPE.itemsize == C.sizeof(StepStats)


def fciqmc_step(run: Run, n_steps: int = 1, as_array: bool = False):
    """Advance n_steps; returns a list of per-step stats dicts, or with
    as_array a numpy structured array over the same memory (no per-step
    Python work)."""
    arr = (StepStats * max(1, n_steps))()
    _check(lib().fciqmc_step(run.handle, int(n_steps), arr))
    if as_array:
        return np.frombuffer(arr, dtype=STATS_DTYPE, count=n_steps)
    return [{k: getattr(arr[i], k) for k, _ in StepStats._fields_} for i in range(n_steps)]


class Pair:
    """Two replicas stepped in lockstep (replica-pair PT2 correction)."""

    def __init__(self, handle, runs):
        self.handle = handle
        self.runs = runs  # keep both runs alive

    def free(self):
        if self.handle:
            lib().fciqmc_pair_free(self.handle)
            self.handle = None


def fciqmc_pair_create(run1: Run, run2: Run) -> Pair:
    h = C.c_void_p()
    _check(lib().fciqmc_pair_create(run1.handle, run2.handle, C.byref(h)))
    return Pair(h, (run1, run2))


def fciqmc_pair_step(pair: Pair, n_steps: int = 1):
    """n_steps lockstep steps: (stats of replica 1, stats of replica 2, dE2
    of each step, normalised by that step's replica overlap, as a numpy
    array; NaN where a step was not evaluated)."""
    a1 = (StepStats * max(1, n_steps))()
    a2 = (StepStats * max(1, n_steps))()
    d = np.zeros(max(1, n_steps))
    _check(lib().fciqmc_pair_step(pair.handle, int(n_steps), a1, a2, _p(d, C.c_double)))
    conv = lambda arr: [{k: getattr(arr[i], k) for k, _ in StepStats._fields_} for i in range(n_steps)]
    return conv(a1), conv(a2), d[:n_steps]


def fciqmc_pair_pt2(pair: Pair, skip: int = 0) -> dict:
    m, e, n = C.c_double(), C.c_double(), C.c_int64()
    _check(lib().fciqmc_pair_pt2(pair.handle, int(skip), C.byref(m), C.byref(e), C.byref(n)))
    return {"mean": m.value, "err": e.value, "n": n.value}


def fciqmc_pair_rdm_enable(pair: Pair, on: bool = True):
    _check(lib().fciqmc_pair_rdm_enable(pair.handle, int(bool(on))))


def fciqmc_pair_rdm(pair: Pair, matrix: bool = True) -> dict:
    """The accumulated replica 2-RDM (hermitian, M x M, or None), the
    variational energy, the norm and the steps sampled."""
    dim, steps = C.c_int64(), C.c_int64()
    e, nm = C.c_double(), C.c_double()
    _check(lib().fciqmc_pair_rdm(pair.handle, None, 0, C.byref(dim), None, None, None))
    M = dim.value
    G = np.zeros((M, M)) if matrix else None
    _check(lib().fciqmc_pair_rdm(pair.handle, _p(G, C.c_double) if matrix else None, M * M if matrix else 0,
                                 C.byref(dim), C.byref(e), C.byref(nm), C.byref(steps)))
    return {"gamma": G, "e_var": e.value, "norm": nm.value, "steps": steps.value, "dim": M}


def fciqmc_pair_free(pair: Pair):
    pair.free()


def fciqmc_get_reference(run: Run):
    """(alpha, beta, H_PP + e_core) of the projected energy's reference."""
    a, b, e = C.c_uint64(), C.c_uint64(), C.c_double()
    _check(lib().fciqmc_get_reference(run.handle, C.byref(a), C.byref(b), C.byref(e)))
    return a.value, b.value, e.value


def fciqmc_energy(run: Run) -> dict:
    r = EnergyReport()
    _check(lib().fciqmc_energy(run.handle, C.byref(r)))
    return {k: getattr(r, k) for k, _ in EnergyReport._fields_}


def fciqmc_get_walkers(run: Run):
    """Returns (alpha_masks, beta_masks, values) as numpy arrays."""
    n = C.c_int64()
    rc = lib().fciqmc_get_walkers(run.handle, None, None, 0, C.byref(n))
    if rc not in (0, EOVERFLOW):
        _check(rc)
    cap = max(1, n.value)
    dets = np.zeros(2 * cap, dtype=np.uint64)
    vals = np.zeros(cap, dtype=np.float64)
    _check(lib().fciqmc_get_walkers(run.handle, _p(dets, C.c_uint64), _p(vals, C.c_double), cap,
                                    C.byref(n)))
    m = n.value
    return dets[0:2 * m:2].copy(), dets[1:2 * m:2].copy(), vals[:m].copy()


def fciqmc_set_walkers(run: Run, alpha, beta, vals):
    a = np.asarray(alpha, dtype=np.uint64)
    b = np.asarray(beta, dtype=np.uint64)
    d = np.ascontiguousarray(np.stack([a, b], axis=1).reshape(-1))
    v = np.ascontiguousarray(vals, dtype=np.float64)
    _check(lib().fciqmc_set_walkers(run.handle, _p(d, C.c_uint64), _p(v, C.c_double), len(v)))


def fciqmc_set_core(run: Run, n_core: int) -> int:
    """Semi-stochastic projection: the n_core most populated determinants
    become the deterministic space; returns its size."""
    n = C.c_int64(0)
    _check(lib().fciqmc_set_core(run.handle, int(n_core), C.byref(n)))
    return n.value


def fciqmc_get_core(run: Run):
    """(alpha masks, beta masks, nonzeros of H^D) of the deterministic space."""
    n, nnz = C.c_int64(0), C.c_int64(0)
    _check(lib().fciqmc_get_core(run.handle, None, 0, C.byref(n), C.byref(nnz)))
    d = np.zeros(2 * max(n.value, 1), dtype=np.uint64)
    _check(lib().fciqmc_get_core(run.handle, _p(d, C.c_uint64), n.value, None, None))
    d = d[:2 * n.value].reshape(-1, 2)
    return d[:, 0].copy(), d[:, 1].copy(), nnz.value


def fciqmc_get_core_row(run: Run, k: int):
    """(column indices into D, H_kj) of row k of H^D, in the library's order."""
    n = C.c_int64(0)
    _check(lib().fciqmc_get_core_row(run.handle, int(k), None, None, 0, C.byref(n)))
    cols = np.zeros(max(n.value, 1), dtype=np.int32)
    vals = np.zeros(max(n.value, 1), dtype=np.float64)
    _check(lib().fciqmc_get_core_row(run.handle, int(k), _p(cols, C.c_int32), _p(vals, C.c_double), n.value, None))
    return cols[:n.value].copy(), vals[:n.value].copy()


def fciqmc_get_checkpoint(run: Run) -> dict:
    c = Checkpoint()
    _check(lib().fciqmc_get_checkpoint(run.handle, C.byref(c)))
    return {k: getattr(c, k) for k, _ in Checkpoint._fields_}


def fciqmc_set_checkpoint(run: Run, iter, shift, vary_shift, last_update_iter, last_update_nw):
    c = Checkpoint(int(iter), float(shift), int(vary_shift), int(last_update_iter),
                   float(last_update_nw))
    _check(lib().fciqmc_set_checkpoint(run.handle, C.byref(c)))


def fciqmc_matrix_elements(system: System, dets_i, dets_j) -> np.ndarray:
    """dets_i, dets_j: (n, 2) uint64 arrays of (alpha, beta) masks."""
    di = np.ascontiguousarray(dets_i, dtype=np.uint64).reshape(-1)
    dj = np.ascontiguousarray(dets_j, dtype=np.uint64).reshape(-1)
    n = len(di) // 2
    out = np.zeros(max(n, 1))
    _check(lib().fciqmc_matrix_elements(system.handle, _p(di, C.c_uint64), _p(dj, C.c_uint64), n,
                                        _p(out, C.c_double)))
    return out[:n]


def fciqmc_matrix_elements_noalloc(system: System, dets_i, dets_j) -> np.ndarray:
    """As fciqmc_matrix_elements, staged in the library's fixed device array
    (no device allocation; at most 65536 pairs)."""
    di = np.ascontiguousarray(dets_i, dtype=np.uint64).reshape(-1)
    dj = np.ascontiguousarray(dets_j, dtype=np.uint64).reshape(-1)
    n = len(di) // 2
    out = np.zeros(max(n, 1))
    _check(lib().fciqmc_matrix_elements_noalloc(system.handle, _p(di, C.c_uint64), _p(dj, C.c_uint64), n,
                                                _p(out, C.c_double)))
    return out[:n]


def fciqmc_pchb_row(system: System, opp: bool, row: int, n_orb: int):
    """(prob, alias, weight, row sum) of one heat-bath alias-table row."""
    K = n_orb * n_orb if opp else n_orb * (n_orb - 1) // 2
    prob = np.zeros(K)
    alias = np.zeros(K, dtype=np.int32)
    weight = np.zeros(K)
    tot = C.c_double()
    _check(lib().fciqmc_pchb_row(system.handle, int(bool(opp)), int(row), _p(prob, C.c_double),
                                 _p(alias, C.c_int32), _p(weight, C.c_double), C.byref(tot)))
    return prob, alias, weight, tot.value


def fciqmc_run_device_bytes(run: Run) -> int:
    return int(lib().fciqmc_run_device_bytes(run.handle))


KERNELS = ("spawn", "annihilate", "post")


def fciqmc_profile(run: Run, enable: bool = True):
    """Enable per-kernel event timing; returns (ms per kernel dict, steps, layout)."""
    ms = np.zeros(len(KERNELS))
    steps = C.c_int64()
    layout = np.zeros(2, dtype=np.int64)
    _check(lib().fciqmc_profile(run.handle, int(enable), _p(ms, C.c_double), C.byref(steps),
                                _p(layout, C.c_int64)))
    return dict(zip(KERNELS, ms.tolist())), steps.value, {"buckets": int(layout[0]),
                                                           "spawn_capacity": int(layout[1])}


def fciqmc_free_run(run: Run):
    run.free()


def fciqmc_free_system(system: System):
    system.free()


def fciqmc_batch_create(stream=None) -> Batch:
    out = C.c_void_p()
    _check(lib().fciqmc_batch_create(_stream_ptr(stream), C.byref(out)))
    return Batch(out.value)


def fciqmc_batch_add(batch: Batch, run: Run):
    _check(lib().fciqmc_batch_add(batch.handle, run.handle))
    batch.members.append(run)
    run.batch = batch


def fciqmc_batch_remove(batch: Batch, run: Run):
    _check(lib().fciqmc_batch_remove(batch.handle, run.handle))
    batch.members.remove(run)
    run.batch = None


def fciqmc_batch_size(batch: Batch) -> int:
    return int(lib().fciqmc_batch_size(batch.handle))


def fciqmc_batch_step(batch: Batch, n_steps: int = 1, as_array: bool = False):
    """Advance every member n_steps; returns [step][member] stats dicts, or
    with as_array a (n_steps, members) numpy structured array."""
    m = len(batch.members)
    arr = (StepStats * max(1, n_steps * m))()
    _check(lib().fciqmc_batch_step(batch.handle, int(n_steps), arr))
    if as_array:
        return np.frombuffer(arr, dtype=STATS_DTYPE, count=n_steps * m).reshape(n_steps, m)
    return [[{k: getattr(arr[s * m + i], k) for k, _ in StepStats._fields_} for i in range(m)]
            for s in range(n_steps)]


def fciqmc_batch_tune(batch: Batch, trial_steps: int = 20) -> dict:
    r = TuneReport()
    _check(lib().fciqmc_batch_tune(batch.handle, int(trial_steps), C.byref(r)))
    return {k: getattr(r, k) for k, _ in TuneReport._fields_}


def fciqmc_batch_set_persistent(batch: Batch, on: bool = True):
    _check(lib().fciqmc_batch_set_persistent(batch.handle, int(bool(on))))


def fciqmc_batch_profile(batch: Batch, enable: bool = True):
    """Enable batch kernel timing; returns (ms per kernel dict, batch steps timed)."""
    ms = np.zeros(len(KERNELS))
    steps = C.c_int64()
    _check(lib().fciqmc_batch_profile(batch.handle, int(enable), _p(ms, C.c_double), C.byref(steps)))
    return dict(zip(KERNELS, ms.tolist())), steps.value


def fciqmc_batch_free(batch: Batch):
    batch.free()


def fciqmc_estimate_bytes(system: System, params: Params) -> int:
    n = int(lib().fciqmc_estimate_bytes(system.handle, C.byref(params)))
    if n < 0:
        _check(n)
    return n


class Server:
    def __init__(self, handle):
        self.handle = handle
        self.systems = []  # systems of submitted requests stay alive with the server

    def free(self):
        if self.handle:
            lib().fciqmc_server_free(self.handle)
            self.handle = None


def fciqmc_server_create(hbm_budget_bytes: int, max_running: int = 256, stream=None) -> Server:
    out = C.c_void_p()
    _check(lib().fciqmc_server_create(int(hbm_budget_bytes), int(max_running), _stream_ptr(stream),
                                      C.byref(out)))
    return Server(out.value)


def fciqmc_server_submit(server: Server, system: System, params: Params, check_interval: int = 100,
                         max_steps: int = 100000, t_arrival: float = -1.0) -> int:
    t = C.c_int64()
    _check(lib().fciqmc_server_submit(server.handle, system.handle, C.byref(params),
                                      int(check_interval), int(max_steps), float(t_arrival),
                                      C.byref(t)))
    server.systems.append(system)
    return t.value


def fciqmc_server_poll(server: Server, n_steps: int = 1):
    """Admit and advance; returns (running, queued)."""
    r, q = C.c_int(), C.c_int()
    _check(lib().fciqmc_server_poll(server.handle, int(n_steps), C.byref(r), C.byref(q)))
    return r.value, q.value


def fciqmc_server_info(server: Server, ticket: int) -> dict:
    i = RequestInfo()
    _check(lib().fciqmc_server_info(server.handle, int(ticket), C.byref(i)))
    d = {k: getattr(i, k) for k, _ in RequestInfo._fields_ if k != "energy"}
    d["energy"] = {k: getattr(i.energy, k) for k, _ in EnergyReport._fields_}
    return d


def fciqmc_server_clock(server: Server) -> float:
    return float(lib().fciqmc_server_clock(server.handle))


def fciqmc_server_free(server: Server):
    server.free()
