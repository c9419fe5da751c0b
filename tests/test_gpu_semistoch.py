"""GPU parity of the semi-stochastic projection (Sec. "Semi-stochastic
FCIQMC") against the oracle.  Real coefficients: the deterministic product
and the spawned amplitudes are summed in another order on the GPU, so values
agree to rounding and the surviving determinants agree exactly (no rounding
decision of these seeds sits within an ulp of its threshold)."""
import numpy as np
import pytest

from paper_2006_14956_amd import fciqmc as F
from paper_2006_14956_amd import inputs
from tests import brute
from tests.gpu_helpers import assert_same_walkers, make_gpu_run, make_pair, ref_of

pytestmark = pytest.mark.gpu


def _same_core(run, orun):
    ga, gb, nnz = F.fciqmc_get_core(run)
    oa, ob = orun.core()
    assert np.array_equal(ga, oa) and np.array_equal(gb, ob)
    return len(ga), nnz


def _close_steps(g, o, rtol):
    for gg, oo in zip(g, o):
        assert gg["ndets"] == oo["ndets"] and gg["spawns"] == oo["spawns"]
        assert gg["attempts"] == oo["attempts"]
        assert abs(gg["nw"] - oo["nw"]) <= rtol * oo["nw"]
        assert abs(gg["shift"] - oo["shift"]) <= rtol * max(1.0, abs(oo["shift"]))


def test_deterministic_space_steps():
    """A random population of 400 determinants on a 10-orbital molecule, the
    60 most populated made deterministic (initiator rule on): the chosen
    space, then one step and ten more agree with the oracle."""
    s = inputs.synthetic_molecule(10, 4, 4, seed=2)
    sysd, run, orun = make_pair(s, tau=0.02, target=1e9, mode="real", seed=4, n_a=2.0)
    ra, rb = ref_of(s)
    a, b, v = inputs.random_walker_state(10, 4, 4, 400, seed=5, max_pop=10, integer=False,
                                         include=(ra, rb))
    F.fciqmc_set_walkers(run, a, b, v)
    orun.set_walkers(a, b, v)
    assert F.fciqmc_set_core(run, 60) == 60
    assert orun.set_core(60) == 60
    n, nnz = _same_core(run, orun)
    assert nnz > 0
    _close_steps(F.fciqmc_step(run, 1), orun.step(1), 1e-12)
    assert_same_walkers(run, orun, exact=False, rtol=1e-12)
    _close_steps(F.fciqmc_step(run, 10), orun.step(10), 1e-11)
    assert_same_walkers(run, orun, exact=False, rtol=1e-10)
    F.fciqmc_free_run(run)
    F.fciqmc_free_system(sysd)


def test_whole_space_deterministic():
    """Every determinant of a 100-determinant space deterministic: one step
    is the dense projector applied to C (checked against the oracle and the
    dense matrix), with no stochastic spawn surviving."""
    s = inputs.synthetic_molecule(5, 2, 2, seed=21, rank=8)
    dets = brute.basis(5, 2, 2)
    sysd, run, orun = make_pair(s, tau=0.05, target=1e12, mode="real", seed=3, n_a=3.0)
    rng = np.random.default_rng(2)
    C0 = rng.normal(0.0, 3.0, size=len(dets))
    a = np.array([d[0] for d in dets], dtype=np.uint64)
    b = np.array([d[1] for d in dets], dtype=np.uint64)
    F.fciqmc_set_walkers(run, a, b, C0)
    orun.set_walkers(a, b, C0)
    assert F.fciqmc_set_core(run, 1000) == len(dets)
    orun.set_core(1000)
    _same_core(run, orun)
    g = F.fciqmc_step(run, 1)
    o = orun.step(1)
    _close_steps(g, o, 1e-12)
    assert g[0]["ndets"] == len(dets)
    assert_same_walkers(run, orun, exact=False, rtol=1e-12)
    F.fciqmc_free_run(run)
    F.fciqmc_free_system(sysd)


def test_deterministic_space_survives_store_growth():
    """Grown from the reference with two buckets, so the store doubles while
    the space is active (every re-import re-marks it): 40 steps agree."""
    s = inputs.molecule_8o8e()
    sysd, run, orun = make_pair(s, tau=0.01, target=1e9, mode="real", seed=6, buckets_log2=1,
                                n_initial=50.0)
    g = F.fciqmc_step(run, 30)
    o = orun.step(30)
    _close_steps(g, o, 1e-11)
    assert F.fciqmc_set_core(run, 20) == 20
    orun.set_core(20)
    _same_core(run, orun)
    g = F.fciqmc_step(run, 40)
    o = orun.step(40)
    _close_steps(g, o, 1e-10)
    assert_same_walkers(run, orun, exact=False, rtol=1e-9)
    assert F.fciqmc_profile(run, False)[2]["buckets"] > 2
    F.fciqmc_free_run(run)
    F.fciqmc_free_system(sysd)


def test_deterministic_space_rules():
    """Integer runs refuse a deterministic space, a run that has one cannot
    join a batch, and setting a new population removes it."""
    s = inputs.molecule_8o8e()
    sysd, run, orun = make_pair(s, tau=0.01, target=1e9, mode="integer", seed=1)
    F.fciqmc_step(run, 5)
    with pytest.raises(F.FciqmcError):
        F.fciqmc_set_core(run, 10)
    F.fciqmc_free_run(run)
    _, run2, _ = make_pair(s, tau=0.01, target=1e9, mode="real", seed=1)
    F.fciqmc_step(run2, 5)
    assert F.fciqmc_set_core(run2, 5) == 5
    batch = F.fciqmc_batch_create()
    with pytest.raises(F.FciqmcError):
        F.fciqmc_batch_add(batch, run2)
    F.fciqmc_batch_free(batch)
    a, b, v = F.fciqmc_get_walkers(run2)
    F.fciqmc_set_walkers(run2, a, b, v)
    assert F.fciqmc_get_core(run2)[0].size == 0
    F.fciqmc_free_run(run2)
    F.fciqmc_free_system(sysd)


def _space_population(s, n_orb, na, nb, seed):
    """Every determinant of the space, with seeded real coefficients whose
    magnitudes are distinct (so the n most populated are unambiguous)."""
    dets = brute.basis(n_orb, na, nb)
    a = np.array([d[0] for d in dets], dtype=np.uint64)
    b = np.array([d[1] for d in dets], dtype=np.uint64)
    rng = np.random.default_rng(seed)
    v = 0.5 + 10.0 * rng.permutation(len(dets)).astype(np.float64) / len(dets)
    v *= rng.choice([-1.0, 1.0], size=len(dets))
    return a, b, v


def _oracle_row(osys, ca, cb, k):
    """Row k of H^D from the oracle: (column indices, values) of its nonzeros."""
    h = osys.hij_row(ca[k], cb[k], ca, cb)
    j = np.nonzero(h)[0]
    return j, h[j]


def _gpu_row(run, k):
    c, v = F.fciqmc_get_core_row(run, k)
    o = np.argsort(c, kind="stable")
    return c[o].astype(np.int64), v[o]


def test_hd_rows_equal_the_oracle_whole_space():
    """Every row of H^D over the whole 3136-determinant space of an 8-orbital
    molecule (3 alpha, 3 beta): the columns and values found from removal
    keys are those of the oracle's all-pairs matrix, bit for bit."""
    import oracle
    s = inputs.synthetic_molecule(8, 3, 3, seed=31)
    sysd, run = make_gpu_run(s, tau=0.01, target=1e12, mode="real", seed=1)
    a, b, v = _space_population(s, 8, 3, 3, seed=4)
    F.fciqmc_set_walkers(run, a, b, v)
    assert F.fciqmc_set_core(run, len(a)) == len(a)
    ca, cb, nnz = F.fciqmc_get_core(run)
    osys = oracle.System.from_inputs(s, words=1)
    total = 0
    for k in range(len(ca)):
        gj, gv = _gpu_row(run, k)
        oj, ov = _oracle_row(osys, ca, cb, k)
        assert np.array_equal(gj, oj), k
        assert np.array_equal(gv, ov), k
        total += len(oj)
    assert nnz == total
    F.fciqmc_free_run(run)
    F.fciqmc_free_system(sysd)


def test_hd_beyond_the_all_pairs_size():
    """A deterministic space of 300000 determinants (the 12-orbital, 5+5
    electron space has 627264), twice the largest the all-pairs construction
    took: the space is the 300000 largest |C|, and sampled rows of H^D (the
    first, the last and 40 seeded ones) equal the oracle's bit for bit."""
    import oracle
    s = inputs.synthetic_molecule(12, 5, 5, seed=37)
    sysd, run = make_gpu_run(s, tau=0.01, target=1e12, mode="real", seed=1)
    a, b, v = _space_population(s, 12, 5, 5, seed=6)
    F.fciqmc_set_walkers(run, a, b, v)
    n = 300000
    assert F.fciqmc_set_core(run, n) == n
    ca, cb, nnz = F.fciqmc_get_core(run)
    # the space is the n largest |C| (all distinct), ordered by determinant
    top = np.argsort(-np.abs(v), kind="stable")[:n]
    want = sorted(zip(a[top].tolist(), b[top].tolist()))
    assert list(zip(ca.tolist(), cb.tolist())) == want
    osys = oracle.System.from_inputs(s, words=1)
    rows = [0, n - 1] + list(np.random.default_rng(8).choice(n, size=40, replace=False))
    for k in rows:
        gj, gv = _gpu_row(run, int(k))
        oj, ov = _oracle_row(osys, ca, cb, int(k))
        assert np.array_equal(gj, oj), k
        assert np.array_equal(gv, ov), k
    sizes = [F.fciqmc_get_core_row(run, k)[0].size for k in range(0, n, 997)]
    assert all(x > 0 for x in sizes)
    assert nnz > 100 * n
    F.fciqmc_free_run(run)
    F.fciqmc_free_system(sysd)
