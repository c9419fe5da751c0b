"""Shared helpers of the GPU parity tests: run the HIP library and the oracle
side by side on the same seeded inputs and compare."""
import numpy as np

import oracle
from paper_2006_14956_amd import fciqmc as F

GEN = {"uniform": (F.GEN_UNIFORM, oracle.GEN_UNIFORM),
       "lattice": (F.GEN_LATTICE, oracle.GEN_LATTICE),
       "pchb": (F.GEN_PCHB, oracle.GEN_PCHB),
       "cs": (F.GEN_CS, oracle.GEN_CS),
       "pe": (F.GEN_PE, oracle.GEN_PE)}


def ref_of(s):
    if s.ref_alpha or s.ref_beta:
        return int(s.ref_alpha), int(s.ref_beta)
    return (1 << s.n_alpha) - 1, (1 << s.n_beta) - 1


def make_gpu_run(s, tau, target, gen="uniform", n_a=-1.0, mode="integer", seed=1, zeta=0.05,
                 interval=10, c_min=1.0, det_words=0, n_initial=10.0, p_single=-1.0, p_opp=-1.0,
                 buckets_log2=0, max_spawns=0, stream=None, replica=0, sysd=None, max_dets=0,
                 adaptive=0, rechoose=0, ref=None):
    """(system handle, gpu_run) started from n_initial walkers on the reference."""
    g, _ = GEN[gen]
    m = F.MODE_INTEGER if mode == "integer" else F.MODE_REAL
    if sysd is None:
        sysd = F.fciqmc_load_integrals(s.n_orb, s.n_alpha, s.n_beta, s.e_core, s.h1, s.eri)
    ra, rb = ref if ref is not None else ref_of(s)
    p = F.fciqmc_params_default(tau=tau, walker_target=target, initiator_na=n_a, mode=m,
                                excitgen=g, seed=seed, shift_damping=zeta, shift_interval=interval,
                                c_min=c_min, det_words=det_words, n_initial=n_initial,
                                ref_alpha=ra, ref_beta=rb, p_single=p_single, p_opp=p_opp,
                                buckets_log2=buckets_log2, max_spawns=max_spawns,
                                replica_id=replica, max_dets=max_dets, adaptive_shift=adaptive,
                                ref_rechoose=rechoose)
    return sysd, F.fciqmc_init(sysd, p, stream=stream)


def make_pair(s, tau, target, gen="uniform", n_a=-1.0, mode="integer", seed=1, zeta=0.05,
              interval=10, c_min=1.0, det_words=0, n_initial=10.0, p_single=-1.0, p_opp=-1.0,
              buckets_log2=0, max_spawns=0, stream=None, replica=0, max_dets=0, adaptive=0, rechoose=0,
              ref=None):
    """(gpu_run, oracle_run) started from n_initial walkers on the reference."""
    _, o = GEN[gen]
    sysd, run = make_gpu_run(s, tau, target, gen=gen, n_a=n_a, mode=mode, seed=seed, zeta=zeta,
                             interval=interval, c_min=c_min, det_words=det_words,
                             n_initial=n_initial, p_single=p_single, p_opp=p_opp,
                             buckets_log2=buckets_log2, max_spawns=max_spawns, stream=stream,
                             replica=replica, max_dets=max_dets, adaptive=adaptive, rechoose=rechoose,
                             ref=ref)
    ra, rb = ref if ref is not None else ref_of(s)
    words = det_words if det_words else (1 if s.n_orb <= 32 else 2)
    osys = oracle.System.from_inputs(s, words=words)
    orun = oracle.Run(osys, ref=(ra, rb), tau=tau, target=target, n_a=n_a, c_min=c_min,
                      zeta=zeta, p_single=p_single, p_opp=p_opp, interval=interval,
                      mode=oracle.MODE_INTEGER if mode == "integer" else oracle.MODE_REAL,
                      gen=o, seed=seed, replica=replica, adaptive=adaptive, rechoose=rechoose)
    orun.set_walkers([ra], [rb], [n_initial])
    return sysd, run, orun


def sorted_walkers(a, b, v):
    i = np.lexsort((b, a))
    return a[i], b[i], v[i]


def gpu_walkers(run):
    return sorted_walkers(*F.fciqmc_get_walkers(run))


def oracle_walkers(orun):
    a, b, v, _ = orun.get_walkers()
    return sorted_walkers(a, b, v)


def assert_same_walkers(run, orun, exact=True, rtol=0.0):
    ga, gb, gv = gpu_walkers(run)
    oa, ob, ov = oracle_walkers(orun)
    assert len(ga) == len(oa), (len(ga), len(oa))
    assert np.array_equal(ga, oa) and np.array_equal(gb, ob)
    if exact:
        assert np.array_equal(gv, ov), np.max(np.abs(gv - ov))
    else:
        assert np.allclose(gv, ov, rtol=rtol, atol=0.0), np.max(np.abs(gv - ov) / np.abs(ov))


def enum_tol(x):
    # estimator sums run in different orders on the two sides: their fp64
    # rounding stays many orders of magnitude below 1e-10 relative
    return 1e-10 * max(1.0, abs(x))


def assert_same_stats(g, o, exact_shift=True):
    for k in ("nw", "nref", "ndets", "attempts", "spawns"):
        assert g[k] == o[k], (k, g[k], o[k], g, o)
    assert g["vary_shift"] == o["vary"]
    if exact_shift:
        assert g["shift"] == o["shift"], (g["shift"], o["shift"])
    assert abs(g["enum_"] - o["enum_"]) <= enum_tol(o["enum_"]), (g["enum_"], o["enum_"])


def assert_same_gpu_stats(a, b):
    """Two GPU runs of the same population: every count and the shift agree
    exactly; the E_proj numerator to the reordered-sum bound (the LDS hash
    order of a bucket may differ between launches)."""
    for k in ("nw", "nref", "ndets", "attempts", "spawns", "vary_shift", "shift", "iter"):
        assert a[k] == b[k], (k, a[k], b[k])
    assert abs(a["enum_"] - b["enum_"]) <= enum_tol(b["enum_"]), (a["enum_"], b["enum_"])


def assert_same_gpu_walkers(r1, r2, exact=True, rtol=0.0):
    a1, b1, v1 = gpu_walkers(r1)
    a2, b2, v2 = gpu_walkers(r2)
    assert len(a1) == len(a2), (len(a1), len(a2))
    assert np.array_equal(a1, a2) and np.array_equal(b1, b2)
    if exact:
        assert np.array_equal(v1, v2)
    else:
        assert np.allclose(v1, v2, rtol=rtol, atol=0.0)


def solve_alone(sysd, params, interval, max_steps):
    """The plain path of one solve: step the run alone, check its energy
    report every `interval` steps, stop when converged or at max_steps.
    Returns (steps, attempts, energy report)."""
    run = F.fciqmc_init(sysd, params)
    steps, att = 0, 0
    while True:
        n = min(interval - steps % interval, max_steps - steps)
        st = F.fciqmc_step(run, n)
        steps += n
        att += sum(x["attempts"] for x in st)
        e = F.fciqmc_energy(run)
        if e["converged"] or steps >= max_steps:
            break
    F.fciqmc_free_run(run)
    return steps, att, e


def assert_same_report(a, b):
    """Energy reports of the same trajectory: shift statistics exact, the
    projected energy to the reordered-sum bound of its numerator."""
    for k in ("shift", "shift_err", "e_ref", "n_samples", "first_step", "steps_done", "converged"):
        assert a[k] == b[k] or (a[k] != a[k] and b[k] != b[k]), (k, a[k], b[k])
    for k in ("e_proj", "e_proj_err"):
        assert abs(a[k] - b[k]) <= 1e-8 * max(1.0, abs(b[k])) or (a[k] != a[k] and b[k] != b[k]), (k, a[k], b[k])
