"""CPU oracle for the FCIQMC step -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  It wraps ``fciqmc_oracle.c`` (plain C, FP64, no FMA
contraction) through ctypes and shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fciqmc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MODE_INTEGER, MODE_REAL = 0, 1
GEN_UNIFORM, GEN_LATTICE, GEN_PCHB, GEN_CS, GEN_PE = 0, 1, 2, 3, 4


def build(force: bool = True) -> str:
    """Compile the oracle to ``oracle/liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        u64, i64, dbl, vp = C.c_uint64, C.c_int64, C.c_double, C.c_void_p
        pu64, pdbl, pint = C.POINTER(u64), C.POINTER(dbl), C.POINTER(C.c_int)
        pu32 = C.POINTER(C.c_uint32)
        L.orc_philox4x32_10.argtypes = [pu32, pu32, pu32]
        L.orc_sys_create.restype = vp
        L.orc_sys_create.argtypes = [C.c_int, C.c_int, C.c_int, dbl, pdbl, pdbl]
        L.orc_sys_set_words.argtypes = [vp, C.c_int]
        L.orc_sys_free.argtypes = [vp]
        L.orc_hdiag.restype = dbl
        L.orc_hdiag.argtypes = [vp, u64, u64]
        L.orc_hij.restype = dbl
        L.orc_hij.argtypes = [vp, u64, u64, u64, u64]
        L.orc_hij_row.restype = None
        L.orc_hij_row.argtypes = [vp, u64, u64, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.c_int64,
                                  C.POINTER(dbl)]
        L.orc_uniform_apply_flat.argtypes = [vp, u64, u64, C.c_int, u64, u64, dbl, pu64, pu64, pdbl]
        L.orc_uniform_count2_flat.restype = u64
        L.orc_uniform_count2_flat.argtypes = [vp, u64, u64, C.c_int, u64]
        L.orc_lattice_apply_flat.argtypes = [vp, u64, u64, u64, u64, pu64, pu64, pdbl]
        L.orc_lattice_degree.argtypes = [vp, C.c_int]
        L.orc_pchb_build.argtypes = [vp]
        L.orc_pchb_row.argtypes = [vp, C.c_int, C.c_int, pdbl, pdbl, pint, pdbl]
        L.orc_layout.argtypes = [vp, u64, u64, pu64, pu64]
        L.orc_unlayout.argtypes = [vp, u64, u64, pu64, pu64]
        L.orc_run_create.restype = vp
        L.orc_run_create.argtypes = [vp, C.POINTER(OrcParams), u64, u64]
        L.orc_run_free.argtypes = [vp]
        L.orc_run_h00.restype = dbl
        L.orc_run_h00.argtypes = [vp]
        L.orc_run_p_single.restype = dbl
        L.orc_run_p_single.argtypes = [vp]
        L.orc_run_set_walkers.argtypes = [vp, pu64, pu64, pdbl, i64]
        L.orc_run_set_state.argtypes = [vp, i64, dbl, C.c_int, i64, dbl]
        L.orc_run_get_state.argtypes = [vp, C.POINTER(i64), pdbl, pint, C.POINTER(i64), pdbl]
        L.orc_run_size.restype = i64
        L.orc_run_size.argtypes = [vp]
        L.orc_run_get_walkers.argtypes = [vp, pu64, pu64, pdbl, pdbl]
        L.orc_run_step.argtypes = [vp, C.POINTER(OrcStats)]
        L.orc_run_estimate.argtypes = [vp, pdbl, pdbl, pdbl]
        L.orc_generate.argtypes = [vp, u64, u64, i64, u64, pu64, pu64, pdbl, pdbl]
        L.orc_run_set_core.restype = i64
        L.orc_run_set_core.argtypes = [vp, i64]
        L.orc_run_core_size.restype = i64
        L.orc_run_core_size.argtypes = [vp]
        L.orc_run_get_core.argtypes = [vp, pu64, pu64]
        L.orc_run_collect_rejected.argtypes = [vp, C.c_int]
        L.orc_pair_pt2.restype = dbl
        L.orc_pair_pt2.argtypes = [vp, vp]
        L.orc_pair_overlap.restype = dbl
        L.orc_pair_overlap.argtypes = [vp, vp]
        L.orc_run_rejected_size.restype = i64
        L.orc_run_rejected_size.argtypes = [vp]
        L.orc_run_get_rejected.argtypes = [vp, pu64, pu64, pdbl]
        L.orc_run_adaptive_f.restype = dbl
        L.orc_run_adaptive_f.argtypes = [vp, u64, u64]
        L.orc_rdm_dim.restype = i64
        L.orc_rdm_dim.argtypes = [vp]
        L.orc_rdm_exact.argtypes = [vp, pu64, pu64, pdbl, pdbl, i64, pdbl]
        L.orc_rdm_energy.restype = dbl
        L.orc_rdm_energy.argtypes = [vp, pdbl, pdbl]
        L.orc_run_log_excitations.argtypes = [vp, C.c_int]
        L.orc_run_excitations.restype = i64
        L.orc_run_excitations.argtypes = [vp]
        L.orc_pair_rdm_step.argtypes = [vp, vp, pdbl]
        L.orc_run_get_proj.argtypes = [vp, pu64, pu64]
        _lib = L
    return _lib


class OrcParams(C.Structure):
    _fields_ = [("tau", C.c_double), ("target", C.c_double), ("n_a", C.c_double),
                ("c_min", C.c_double), ("zeta", C.c_double), ("p_single", C.c_double),
                ("p_opp", C.c_double), ("interval", C.c_int), ("mode", C.c_int),
                ("gen", C.c_int), ("seed", C.c_uint64), ("replica", C.c_uint64),
                ("xi", C.c_double), ("adaptive", C.c_int), ("rechoose", C.c_int)]


class OrcStats(C.Structure):
    _fields_ = [("nw", C.c_double), ("nref", C.c_double), ("enum_", C.c_double),
                ("shift", C.c_double), ("ndets", C.c_int64), ("attempts", C.c_int64),
                ("spawns", C.c_int64), ("vary", C.c_int), ("bloom", C.c_int)]


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def philox4x32_10(counter, key):
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(out, C.c_uint32))
    return out


class System:
    """Integrals held by the oracle (dense N^4 copy of the packed tensor)."""

    def __init__(self, n_orb, n_alpha, n_beta, e_core, h1, eri, words=None):
        self.n_orb, self.n_alpha, self.n_beta, self.e_core = n_orb, n_alpha, n_beta, e_core
        h = np.ascontiguousarray(h1, dtype=np.float64)
        e = np.ascontiguousarray(eri, dtype=np.float64)
        self._h = h
        self._e = e
        self.ptr = lib().orc_sys_create(n_orb, n_alpha, n_beta, float(e_core),
                                        _p(h, C.c_double), _p(e, C.c_double))
        self.words = words if words is not None else (1 if n_orb <= 32 else 2)
        lib().orc_sys_set_words(self.ptr, self.words)
        self._pchb = False

    @classmethod
    def from_inputs(cls, s, words=None):
        return cls(s.n_orb, s.n_alpha, s.n_beta, s.e_core, s.h1, s.eri, words=words)

    def __del__(self):
        try:
            if getattr(self, "ptr", None):
                lib().orc_sys_free(self.ptr)
                self.ptr = None
        except Exception:
            pass

    def hdiag(self, a, b):
        return lib().orc_hdiag(self.ptr, int(a), int(b))

    def hij(self, a1, b1, a2, b2):
        return lib().orc_hij(self.ptr, int(a1), int(b1), int(a2), int(b2))

    def hij_row(self, ar, br, a, b):
        """<D_row|H|D_j> for every (a[j], b[j]) (0 where D_j = D_row), the
        orientation of the deterministic-space matrix."""
        a = np.ascontiguousarray(a, dtype=np.uint64)
        b = np.ascontiguousarray(b, dtype=np.uint64)
        out = np.zeros(len(a), dtype=np.float64)
        lib().orc_hij_row(self.ptr, int(ar), int(br), _p(a, C.c_uint64), _p(b, C.c_uint64), len(a),
                          _p(out, C.c_double))
        return out

    def build_pchb(self):
        if not self._pchb:
            lib().orc_pchb_build(self.ptr)
            self._pchb = True

    def pchb_row(self, opp: bool, row: int):
        N = self.n_orb
        K = N * N if opp else N * (N - 1) // 2
        w = np.zeros(K)
        pr = np.zeros(K)
        al = np.zeros(K, dtype=np.int32)
        s = C.c_double()
        lib().orc_pchb_row(self.ptr, int(opp), int(row), _p(w, C.c_double), _p(pr, C.c_double),
                           _p(al, C.c_int), C.byref(s))
        return w, pr, al, s.value

    def rdm_dim(self):
        """M = C(2N, 2): the 2-RDM is an M x M matrix over spin-orbital pairs k < l."""
        return int(lib().orc_rdm_dim(self.ptr))

    def rdm_exact(self, a, b, ca, cb):
        """Eq. (FCI2RDM) over one determinant list (ascending) with coefficient
        vectors ca (bra) and cb (ket): an M x M array."""
        a = np.ascontiguousarray(a, dtype=np.uint64)
        b = np.ascontiguousarray(b, dtype=np.uint64)
        ca = np.ascontiguousarray(ca, dtype=np.float64)
        cb = np.ascontiguousarray(cb, dtype=np.float64)
        M = self.rdm_dim()
        G = np.zeros(M * M)
        lib().orc_rdm_exact(self.ptr, _p(a, C.c_uint64), _p(b, C.c_uint64), _p(ca, C.c_double),
                            _p(cb, C.c_double), len(a), _p(G, C.c_double))
        return G.reshape(M, M)

    def rdm_energy(self, G):
        """(energy, norm) of a 2-RDM: <A|H|B>/<A|B> + E_core and <A|B>."""
        G = np.ascontiguousarray(G, dtype=np.float64)
        norm = C.c_double()
        e = lib().orc_rdm_energy(self.ptr, _p(G, C.c_double), C.byref(norm))
        return e, norm.value

    def uniform_count2(self, a, b, single, idx1):
        return int(lib().orc_uniform_count2_flat(self.ptr, int(a), int(b), int(single), int(idx1)))

    def uniform_apply(self, a, b, single, idx1, idx2, p_single):
        ta, tb, pg = C.c_uint64(), C.c_uint64(), C.c_double()
        ok = lib().orc_uniform_apply_flat(self.ptr, int(a), int(b), int(single), int(idx1),
                                          int(idx2), float(p_single), C.byref(ta), C.byref(tb),
                                          C.byref(pg))
        return (ta.value, tb.value, pg.value) if ok else None

    def lattice_degree(self, p):
        return lib().orc_lattice_degree(self.ptr, int(p))

    def lattice_apply(self, a, b, idx1, idx2):
        ta, tb, pg = C.c_uint64(), C.c_uint64(), C.c_double()
        ok = lib().orc_lattice_apply_flat(self.ptr, int(a), int(b), int(idx1), int(idx2),
                                          C.byref(ta), C.byref(tb), C.byref(pg))
        return (ta.value, tb.value, pg.value) if ok else None

    def layout(self, a, b):
        w0, w1 = C.c_uint64(), C.c_uint64()
        lib().orc_layout(self.ptr, int(a), int(b), C.byref(w0), C.byref(w1))
        return w0.value, w1.value

    def unlayout(self, w0, w1):
        a, b = C.c_uint64(), C.c_uint64()
        lib().orc_unlayout(self.ptr, int(w0), int(w1), C.byref(a), C.byref(b))
        return a.value, b.value


DEFAULTS = dict(tau=0.01, target=1e4, n_a=-1.0, c_min=1.0, zeta=0.05, p_single=-1.0,
                p_opp=-1.0, interval=10, mode=MODE_INTEGER, gen=GEN_UNIFORM, seed=1, replica=0,
                xi=-1.0, adaptive=0, rechoose=0)


class Run:
    """One walker population propagated by the oracle."""

    def __init__(self, system: System, ref=(0, 0), **params):
        p = dict(DEFAULTS)
        p.update(params)
        if p["p_opp"] < 0:
            n = system.n_alpha + system.n_beta
            npair = n * (n - 1) // 2
            p["p_opp"] = (system.n_alpha * system.n_beta) / npair if npair else 0.0
        if p["gen"] == GEN_PCHB:
            system.build_pchb()
        self.params = p
        self.system = system
        self._cp = OrcParams(**{k: p[k] for k, _ in OrcParams._fields_})
        self.ptr = lib().orc_run_create(system.ptr, C.byref(self._cp), int(ref[0]), int(ref[1]))

    def __del__(self):
        try:
            if getattr(self, "ptr", None):
                lib().orc_run_free(self.ptr)
                self.ptr = None
        except Exception:
            pass

    @property
    def h00(self):
        return lib().orc_run_h00(self.ptr)

    @property
    def p_single(self):
        return lib().orc_run_p_single(self.ptr)

    def set_walkers(self, a, b, v):
        a = np.ascontiguousarray(a, dtype=np.uint64)
        b = np.ascontiguousarray(b, dtype=np.uint64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        lib().orc_run_set_walkers(self.ptr, _p(a, C.c_uint64), _p(b, C.c_uint64),
                                  _p(v, C.c_double), len(v))

    def set_state(self, t, shift, vary, t_last, nw_last):
        lib().orc_run_set_state(self.ptr, int(t), float(shift), int(vary), int(t_last),
                                float(nw_last))

    def get_state(self):
        t, tl = C.c_int64(), C.c_int64()
        s, nl = C.c_double(), C.c_double()
        v = C.c_int()
        lib().orc_run_get_state(self.ptr, C.byref(t), C.byref(s), C.byref(v), C.byref(tl),
                                C.byref(nl))
        return dict(t=t.value, shift=s.value, vary=v.value, t_last=tl.value, nw_last=nl.value)

    def get_walkers(self):
        n = lib().orc_run_size(self.ptr)
        a = np.zeros(n, dtype=np.uint64)
        b = np.zeros(n, dtype=np.uint64)
        v = np.zeros(n)
        d = np.zeros(n)
        lib().orc_run_get_walkers(self.ptr, _p(a, C.c_uint64), _p(b, C.c_uint64),
                                  _p(v, C.c_double), _p(d, C.c_double))
        return a, b, v, d

    def step(self, n=1):
        out = []
        for _ in range(n):
            st = OrcStats()
            lib().orc_run_step(self.ptr, C.byref(st))
            out.append({k: getattr(st, k) for k, _ in OrcStats._fields_})
        return out

    def estimate(self):
        nw, nr, en = C.c_double(), C.c_double(), C.c_double()
        lib().orc_run_estimate(self.ptr, C.byref(nw), C.byref(nr), C.byref(en))
        return dict(nw=nw.value, nref=nr.value, enum_=en.value)

    def set_core(self, n_core):
        """Deterministic space of the n_core most populated determinants
        (semi-stochastic projection); returns its size (-1 in integer mode)."""
        return lib().orc_run_set_core(self.ptr, int(n_core))

    def core(self):
        n = lib().orc_run_core_size(self.ptr)
        a = np.zeros(n, dtype=np.uint64)
        b = np.zeros(n, dtype=np.uint64)
        lib().orc_run_get_core(self.ptr, _p(a, C.c_uint64), _p(b, C.c_uint64))
        return a, b

    def collect_rejected(self, on=True):
        """Record the discarded spawns of each step (for the PT2 correction)."""
        lib().orc_run_collect_rejected(self.ptr, int(bool(on)))

    def rejected_size(self):
        return lib().orc_run_rejected_size(self.ptr)

    def adaptive_f(self, a, b):
        """Adaptive-shift fraction f of (a, b) in the last step (-1: not occupied)."""
        return lib().orc_run_adaptive_f(self.ptr, int(a), int(b))

    def rejected(self):
        """(alpha, beta, weight) of the last step's discarded targets."""
        n = lib().orc_run_rejected_size(self.ptr)
        a = np.zeros(n, dtype=np.uint64)
        b = np.zeros(n, dtype=np.uint64)
        w = np.zeros(n)
        lib().orc_run_get_rejected(self.ptr, _p(a, C.c_uint64), _p(b, C.c_uint64), _p(w, C.c_double))
        return a, b, w

    def log_excitations(self, on=True):
        """Keep the population each step starts from and every excitation it
        generates (for the replica 2-RDM)."""
        lib().orc_run_log_excitations(self.ptr, int(bool(on)))

    def projection_reference(self):
        """The determinant the projected energy is taken against (alpha, beta)."""
        a, b = C.c_uint64(), C.c_uint64()
        lib().orc_run_get_proj(self.ptr, C.byref(a), C.byref(b))
        return a.value, b.value

    def excitations(self):
        return int(lib().orc_run_excitations(self.ptr))

    def generate(self, a, b, t, k):
        ta, tb, pg, H = C.c_uint64(), C.c_uint64(), C.c_double(), C.c_double()
        ok = lib().orc_generate(self.ptr, int(a), int(b), int(t), int(k), C.byref(ta),
                                C.byref(tb), C.byref(pg), C.byref(H))
        return (ta.value, tb.value, pg.value, H.value) if ok else None


def pair_pt2(r1: Run, r2: Run) -> float:
    """Epstein-Nesbet correction from the spawns both replicas discarded in
    their last step (each must collect its rejected spawns), before the
    division by the replica overlap of the populations the step began from."""
    return lib().orc_pair_pt2(r1.ptr, r2.ptr)


def pair_overlap(r1: Run, r2: Run) -> float:
    """sum_i C_i^1 C_i^2 of the two replicas' current populations."""
    return lib().orc_pair_overlap(r1.ptr, r2.ptr)


def pair_rdm_step(r1: Run, r2: Run, G):
    """Add one paired step's sample of the replica 2-RDM to G (M x M, in
    place); both runs must log their excitations."""
    assert G.flags["C_CONTIGUOUS"] and G.dtype == np.float64
    lib().orc_pair_rdm_step(r1.ptr, r2.ptr, _p(G, C.c_double))
    return G
