"""GPU parity of the replica-pair PT2 correction (Sec. "Perturbative
correction", Eq. (pt2_correction), normalised by the replica overlap)
against the oracle.  Integer walkers: both replicas follow the oracle bit
for bit, the discarded weights and the overlap are sums of integers, and
dE2 differs only by the order of its final sums."""
import math

import numpy as np
import pytest

import oracle
from paper_2006_14956_amd import fciqmc as F
from paper_2006_14956_amd import inputs
from tests.gpu_helpers import assert_same_stats, assert_same_walkers, make_gpu_run, ref_of

pytestmark = pytest.mark.gpu


def _replicas(s, n_a, seed=9, det_words=0):
    gpu, orc = [], []
    sysd = F.fciqmc_load_integrals(s.n_orb, s.n_alpha, s.n_beta, s.e_core, s.h1, s.eri)
    ra, rb = ref_of(s)
    words = det_words if det_words else (1 if s.n_orb <= 32 else 2)
    osys = oracle.System.from_inputs(s, words=words)
    for rep in (0, 1):
        _, run = make_gpu_run(s, tau=0.02, target=1e9, n_a=n_a, seed=seed, replica=rep, sysd=sysd,
                              det_words=det_words)
        o = oracle.Run(osys, ref=(ra, rb), tau=0.02, target=1e9, n_a=n_a, seed=seed, replica=rep)
        o.collect_rejected(True)
        gpu.append(run)
        orc.append(o)
    return sysd, gpu, orc


def _set_state(s, gpu, orc, n_dets):
    ra, rb = ref_of(s)
    a, b, v = inputs.random_walker_state(s.n_orb, s.n_alpha, s.n_beta, n_dets, seed=3, max_pop=30,
                                         include=(ra, rb))
    for g, o in zip(gpu, orc):
        F.fciqmc_set_walkers(g, a, b, v)
        F.fciqmc_set_checkpoint(g, 0, -0.7, 1, 0, float(np.abs(v).sum()))
        o.set_walkers(a, b, v)
        o.set_state(0, -0.7, 1, 0, float(np.abs(v).sum()))


@pytest.mark.parametrize("words", [1, 2])
def test_pair_correction_matches_oracle(words):
    """A random population on a 10-orbital molecule (initiator rule n_a = 3)
    in two replicas: every step's dE2, both replicas' statistics and their
    walker lists agree with the oracle for 12 steps."""
    s = inputs.synthetic_molecule(10, 4, 3, seed=7)
    sysd, gpu, orc = _replicas(s, 3.0, det_words=words)
    _set_state(s, gpu, orc, 300)
    pair = F.fciqmc_pair_create(gpu[0], gpu[1])
    nonzero = 0
    for step in range(12):
        g1, g2, d = F.fciqmc_pair_step(pair, 1)
        ovl = oracle.pair_overlap(orc[0], orc[1])
        o1 = orc[0].step(1)
        o2 = orc[1].step(1)
        assert_same_stats(g1[0], o1[0])
        assert_same_stats(g2[0], o2[0])
        want = oracle.pair_pt2(orc[0], orc[1]) / ovl
        assert not math.isnan(d[0])
        assert abs(d[0] - want) <= 1e-10 * max(1e-12, abs(want)), (step, d[0], want)
        nonzero += want != 0.0
    assert nonzero >= 10
    for g, o in zip(gpu, orc):
        assert_same_walkers(g, o)
    rep = F.fciqmc_pair_pt2(pair)
    assert rep["n"] == 12 and math.isfinite(rep["mean"])
    F.fciqmc_pair_free(pair)
    for g in gpu:
        F.fciqmc_free_run(g)
    F.fciqmc_free_system(sysd)


def test_pair_through_store_growth():
    """Both replicas start on two buckets and grow from 1000 walkers on the
    reference to most of the 4900 determinants, so a store outgrows the
    common bucket count during a step: that step is evaluated with the two
    replicas in different layouts, both stores are then re-bucketed, and
    every step's dE2 equals the oracle's."""
    s = inputs.molecule_8o8e()
    sysd = F.fciqmc_load_integrals(s.n_orb, s.n_alpha, s.n_beta, s.e_core, s.h1, s.eri)
    ra, rb = ref_of(s)
    osys = oracle.System.from_inputs(s)
    gpu, orc = [], []
    for rep in (0, 1):
        _, run = make_gpu_run(s, tau=0.02, target=1e9, n_a=3.0, seed=4, replica=rep, sysd=sysd,
                              buckets_log2=1, n_initial=1000.0)
        o = oracle.Run(osys, ref=(ra, rb), tau=0.02, target=1e9, n_a=3.0, seed=4, replica=rep)
        o.set_walkers([ra], [rb], [1000.0])
        o.collect_rejected(True)
        gpu.append(run)
        orc.append(o)
    pair = F.fciqmc_pair_create(gpu[0], gpu[1])
    grew = 0
    for step in range(120):
        b0 = F.fciqmc_profile(gpu[0], False)[2]["buckets"]
        g1, g2, d = F.fciqmc_pair_step(pair, 1)
        grew += F.fciqmc_profile(gpu[0], False)[2]["buckets"] != b0
        ovl = oracle.pair_overlap(orc[0], orc[1])
        o1 = orc[0].step(1)
        o2 = orc[1].step(1)
        assert_same_stats(g1[0], o1[0])
        assert_same_stats(g2[0], o2[0])
        want = oracle.pair_pt2(orc[0], orc[1]) / ovl
        assert not math.isnan(d[0]), step
        assert abs(d[0] - want) <= 1e-10 * max(1e-12, abs(want)), (step, d[0], want)
    assert grew >= 1
    assert F.fciqmc_profile(gpu[0], False)[2]["buckets"] > 2
    rep = F.fciqmc_pair_pt2(pair)
    assert rep["n"] == 120
    F.fciqmc_pair_free(pair)
    for g in gpu:
        F.fciqmc_free_run(g)
    F.fciqmc_free_system(sysd)


def test_pair_multi_step_calls_through_growth():
    """The growth scenario again, in calls of 7 paired steps: the values a
    call gathers from the device at its end are, step by step, the oracle's
    (also where a store outgrew the common bucket count), and the per-step
    statistics of both replicas agree with it."""
    s = inputs.molecule_8o8e()
    sysd = F.fciqmc_load_integrals(s.n_orb, s.n_alpha, s.n_beta, s.e_core, s.h1, s.eri)
    ra, rb = ref_of(s)
    osys = oracle.System.from_inputs(s)
    gpu, orc = [], []
    for rep in (0, 1):
        _, run = make_gpu_run(s, tau=0.02, target=1e9, n_a=3.0, seed=4, replica=rep, sysd=sysd,
                              buckets_log2=1, n_initial=1000.0)
        o = oracle.Run(osys, ref=(ra, rb), tau=0.02, target=1e9, n_a=3.0, seed=4, replica=rep)
        o.set_walkers([ra], [rb], [1000.0])
        o.collect_rejected(True)
        gpu.append(run)
        orc.append(o)
    pair = F.fciqmc_pair_create(gpu[0], gpu[1])
    evaluated = 0
    for call in range(9):
        g1, g2, d = F.fciqmc_pair_step(pair, 7)
        assert len(d) == 7 and len(g1) == 7 and len(g2) == 7
        for i in range(7):
            ovl = oracle.pair_overlap(orc[0], orc[1])
            o1 = orc[0].step(1)
            o2 = orc[1].step(1)
            assert_same_stats(g1[i], o1[0])
            assert_same_stats(g2[i], o2[0])
            assert not math.isnan(d[i]), (call, i)
            want = oracle.pair_pt2(orc[0], orc[1]) / ovl
            assert abs(d[i] - want) <= 1e-10 * max(1e-12, abs(want)), (call, i, d[i], want)
            evaluated += 1
    assert evaluated == 63
    assert F.fciqmc_profile(gpu[0], False)[2]["buckets"] > 2
    for g, o in zip(gpu, orc):
        assert_same_walkers(g, o)
    assert F.fciqmc_pair_pt2(pair)["n"] == evaluated
    F.fciqmc_pair_free(pair)
    for g in gpu:
        F.fciqmc_free_run(g)
    F.fciqmc_free_system(sysd)


def test_pair_many_discards_per_bucket():
    """Thousands of discarded spawns per bucket: 1000 non-initiators with up
    to 100 walkers each (n_a = 100) on the 8-orbital molecule in eight
    buckets, so a bucket holds several times more discard records than one
    pass of the pair table takes and the sum runs in passes over disjoint
    hash ranges; every step's dE2 equals the oracle's."""
    s = inputs.molecule_8o8e()
    sysd = F.fciqmc_load_integrals(s.n_orb, s.n_alpha, s.n_beta, s.e_core, s.h1, s.eri)
    ra, rb = ref_of(s)
    osys = oracle.System.from_inputs(s)
    gpu, orc = [], []
    for rep in (0, 1):
        _, run = make_gpu_run(s, tau=0.04, target=1e9, n_a=100.0, seed=6, replica=rep, sysd=sysd,
                              buckets_log2=3)
        o = oracle.Run(osys, ref=(ra, rb), tau=0.04, target=1e9, n_a=100.0, seed=6, replica=rep)
        o.collect_rejected(True)
        gpu.append(run)
        orc.append(o)
    a, b, v = inputs.random_walker_state(s.n_orb, s.n_alpha, s.n_beta, 1000, seed=5, max_pop=100,
                                         include=(ra, rb))
    for g, o in zip(gpu, orc):
        F.fciqmc_set_walkers(g, a, b, v)
        F.fciqmc_set_checkpoint(g, 0, -0.7, 1, 0, float(np.abs(v).sum()))
        o.set_walkers(a, b, v)
        o.set_state(0, -0.7, 1, 0, float(np.abs(v).sum()))
    pair = F.fciqmc_pair_create(gpu[0], gpu[1])
    nb = F.fciqmc_profile(gpu[0], False)[2]["buckets"]
    for step in range(3):
        g1, g2, d = F.fciqmc_pair_step(pair, 1)
        ovl = oracle.pair_overlap(orc[0], orc[1])
        o1 = orc[0].step(1)
        o2 = orc[1].step(1)
        assert_same_stats(g1[0], o1[0])
        assert_same_stats(g2[0], o2[0])
        if step == 0:
            # records per bucket far above one pass of the table (768)
            assert g1[0]["spawns"] > 2000 * nb, (g1[0]["spawns"], nb)
        want = oracle.pair_pt2(orc[0], orc[1]) / ovl
        assert want != 0.0
        assert abs(d[0] - want) <= 1e-10 * max(1e-12, abs(want)), (step, d[0], want)
    F.fciqmc_pair_free(pair)
    for g in gpu:
        F.fciqmc_free_run(g)
    F.fciqmc_free_system(sysd)


def test_pair_without_initiator_rule_is_zero():
    """No initiator rule: nothing is discarded and dE2 is 0 every step."""
    s = inputs.synthetic_molecule(10, 4, 3, seed=7)
    sysd, gpu, orc = _replicas(s, -1.0)
    _set_state(s, gpu, orc, 200)
    pair = F.fciqmc_pair_create(gpu[0], gpu[1])
    _, _, d = F.fciqmc_pair_step(pair, 5)
    assert np.all(d == 0.0)
    F.fciqmc_pair_free(pair)
    for g in gpu:
        F.fciqmc_free_run(g)
    F.fciqmc_free_system(sysd)


def test_pair_rules():
    """Replicas need independent streams; a paired run cannot join a batch;
    a pair whose replica was freed refuses to step."""
    s = inputs.molecule_8o8e()
    sysd = F.fciqmc_load_integrals(s.n_orb, s.n_alpha, s.n_beta, s.e_core, s.h1, s.eri)
    _, r1 = make_gpu_run(s, tau=0.01, target=1e4, n_a=3.0, seed=1, replica=0, sysd=sysd)
    _, r2 = make_gpu_run(s, tau=0.01, target=1e4, n_a=3.0, seed=1, replica=0, sysd=sysd)
    with pytest.raises(F.FciqmcError):
        F.fciqmc_pair_create(r1, r2)
    _, r3 = make_gpu_run(s, tau=0.01, target=1e4, n_a=3.0, seed=1, replica=1, sysd=sysd)
    pair = F.fciqmc_pair_create(r1, r3)
    F.fciqmc_pair_step(pair, 20)
    batch = F.fciqmc_batch_create()
    with pytest.raises(F.FciqmcError):
        F.fciqmc_batch_add(batch, r1)
    F.fciqmc_batch_free(batch)
    F.fciqmc_free_run(r3)
    with pytest.raises(F.FciqmcError):
        F.fciqmc_pair_step(pair, 1)
    F.fciqmc_pair_free(pair)
    F.fciqmc_step(r1, 3)   # the surviving run steps alone again
    F.fciqmc_free_run(r1)
    F.fciqmc_free_run(r2)
    F.fciqmc_free_system(sysd)
