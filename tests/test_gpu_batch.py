"""GPU: batched stepping.  Populations advanced together by shared launches
follow exactly the trajectories they follow alone (integer mode: every count,
the shift and the walker lists bit for bit), and the oracle's."""
import pytest

from paper_2006_14956_amd import fciqmc as F
from paper_2006_14956_amd import inputs
from tests.gpu_helpers import (assert_same_gpu_stats, assert_same_gpu_walkers, assert_same_stats,
                               assert_same_walkers, make_gpu_run, make_pair, ref_of)

pytestmark = pytest.mark.gpu

# (system, run options): uneven orbital counts, both determinant widths, all
# five generators, initiator on and off
MEMBERS = [
    (lambda: inputs.molecule_8o8e(), dict(tau=0.01, target=1e4, seed=1)),
    (lambda: inputs.synthetic_molecule(10, 5, 5, seed=3), dict(tau=0.01, target=3e4, n_a=3.0, seed=2)),
    (lambda: inputs.synthetic_molecule(12, 6, 6, seed=5), dict(tau=0.005, target=5e4, seed=3)),
    (lambda: inputs.hubbard_4x4(), dict(tau=0.005, target=2e4, gen="lattice", n_a=3.0, zeta=0.3)),
    (lambda: inputs.synthetic_molecule(10, 4, 3, seed=7), dict(tau=0.01, target=1e4, gen="pchb",
                                                               det_words=2, seed=4)),
    (lambda: inputs.synthetic_molecule(9, 4, 4, seed=11), dict(tau=0.01, target=2e4, gen="pchb",
                                                               n_a=3.0, seed=5)),
    (lambda: inputs.synthetic_molecule(10, 4, 4, seed=13), dict(tau=0.01, target=1e4, gen="cs", seed=6)),
    (lambda: inputs.synthetic_molecule(11, 5, 4, seed=17), dict(tau=0.005, target=2e4, gen="pe",
                                                                n_a=3.0, det_words=2, seed=7)),
]


def _pairs(members):
    """For each member: (system handle, batched run, solo run)."""
    out = []
    for mk, kw in members:
        s = mk()
        sysd, rb = make_gpu_run(s, **kw)
        _, rs = make_gpu_run(s, sysd=sysd, **kw)
        out.append((sysd, rb, rs))
    return out


def _free(pairs, batch=None):
    if batch is not None:
        F.fciqmc_batch_free(batch)
    for sysd, rb, rs in pairs:
        F.fciqmc_free_run(rb)
        F.fciqmc_free_run(rs)
        F.fciqmc_free_system(sysd)


@pytest.mark.parametrize("persistent", [True, False])
def test_batch_members_follow_their_solo_trajectories(persistent):
    """Every member's trajectory in the batch is its solo trajectory, with
    the step as one cooperative launch per group (generator chosen per
    member) or as separate launches per phase."""
    pairs = _pairs(MEMBERS)
    batch = F.fciqmc_batch_create()
    F.fciqmc_batch_set_persistent(batch, persistent)
    for _, rb, _ in pairs:
        F.fciqmc_batch_add(batch, rb)
    assert F.fciqmc_batch_size(batch) == len(MEMBERS)
    for block in range(4):
        bst = F.fciqmc_batch_step(batch, 60)
        for m, (_, _, rs) in enumerate(pairs):
            sst = F.fciqmc_step(rs, 60)
            for s in range(60):
                assert_same_gpu_stats(bst[s][m], sst[s])
        for _, rb, rs in pairs:
            assert_same_gpu_walkers(rb, rs)
    assert all(bst[-1][m]["nw"] > 1000 for m in range(len(MEMBERS)))
    _free(pairs, batch)


def test_batch_member_matches_oracle():
    """8 electrons in 8 orbitals (uniform generator, target 1e4) inside a batch
    with two other molecules: identical to the oracle step by step."""
    s = inputs.molecule_8o8e()
    sysd, run, orun = make_pair(s, tau=0.01, target=1e4, seed=1)
    others = _pairs(MEMBERS[1:3])
    batch = F.fciqmc_batch_create()
    F.fciqmc_batch_add(batch, others[0][1])
    F.fciqmc_batch_add(batch, run)
    F.fciqmc_batch_add(batch, others[1][1])
    for block in range(3):
        bst = F.fciqmc_batch_step(batch, 100)
        o = orun.step(100)
        for s_ in range(100):
            assert_same_stats(bst[s_][1], o[s_])
        assert_same_walkers(run, orun)
    F.fciqmc_batch_free(batch)
    F.fciqmc_free_run(run)
    F.fciqmc_free_system(sysd)
    _free(others)


@pytest.mark.parametrize("persistent", [True, False])
def test_capacity_growth_inside_a_batch(persistent):
    """A member with two buckets and a 100-record spawn buffer overflows and
    replays its steps alone; neither it nor its neighbour changes trajectory."""
    s = inputs.molecule_8o8e()
    kw = dict(tau=0.01, target=1e4, seed=3, buckets_log2=1, max_spawns=100)
    sysd, rb = make_gpu_run(s, **kw)
    _, rs = make_gpu_run(s, sysd=sysd, **kw)
    other = _pairs(MEMBERS[2:3])
    batch = F.fciqmc_batch_create()
    F.fciqmc_batch_set_persistent(batch, persistent)
    F.fciqmc_batch_add(batch, rb)
    F.fciqmc_batch_add(batch, other[0][1])
    bst = F.fciqmc_batch_step(batch, 200)
    sst = F.fciqmc_step(rs, 200)
    ost = F.fciqmc_step(other[0][2], 200)
    for i in range(200):
        assert_same_gpu_stats(bst[i][0], sst[i])
        assert_same_gpu_stats(bst[i][1], ost[i])
    assert sum(x[0]["retries"] for x in bst) > 0
    assert_same_gpu_walkers(rb, rs)
    assert_same_gpu_walkers(other[0][1], other[0][2])
    F.fciqmc_batch_free(batch)
    F.fciqmc_free_run(rb)
    F.fciqmc_free_run(rs)
    F.fciqmc_free_system(sysd)
    _free(other)


def test_single_generator_persistent_batch():
    """Twelve uniform-generator molecules of 8 to 14 orbitals (the fixed-
    generator form of the cooperative launch): each member equals its solo
    run after 300 steps, and the persistent and per-phase forms give the same
    populations."""
    members = [(lambda n=n, i=i: inputs.synthetic_molecule(n, n // 2, n // 2, seed=40 + i),
                dict(tau=0.004, target=5e3 * (1 + i % 4), seed=10 + i))
               for i, n in enumerate([8, 9, 10, 11, 12, 13, 14, 8, 10, 12, 9, 11])]
    pairs = _pairs(members)
    batch = F.fciqmc_batch_create()
    F.fciqmc_batch_set_persistent(batch, True)
    for _, rb, _ in pairs:
        F.fciqmc_batch_add(batch, rb)
    bst = F.fciqmc_batch_step(batch, 150)
    F.fciqmc_batch_set_persistent(batch, False)
    bst += F.fciqmc_batch_step(batch, 50)
    F.fciqmc_batch_set_persistent(batch, True)
    bst += F.fciqmc_batch_step(batch, 100)
    for m, (_, rb, rs) in enumerate(pairs):
        sst = F.fciqmc_step(rs, 300)
        for s_ in range(300):
            assert_same_gpu_stats(bst[s_][m], sst[s_])
        assert_same_gpu_walkers(rb, rs)
    assert all(bst[-1][m]["nw"] > 1000 for m in range(len(members)))
    _free(pairs, batch)


def test_tuning_keeps_trajectories():
    """The autotuner re-partitions the walker stores and changes launch grids
    while stepping; the members' trajectories are those of solo runs."""
    pairs = _pairs(MEMBERS[:4])
    batch = F.fciqmc_batch_create()
    for _, rb, _ in pairs:
        F.fciqmc_batch_add(batch, rb)
    F.fciqmc_batch_step(batch, 150)
    rep = F.fciqmc_batch_tune(batch, trial_steps=4)
    assert rep["trials"] >= 4 and rep["steps"] == 4 * rep["trials"]
    assert rep["rate_best"] >= rep["rate_initial"] > 0
    bst = F.fciqmc_batch_step(batch, 40)
    n = 150 + rep["steps"] + 40
    for m, (_, rb, rs) in enumerate(pairs):
        sst = F.fciqmc_step(rs, n)
        assert_same_gpu_stats(bst[-1][m], sst[-1])
        assert_same_gpu_walkers(rb, rs)
    _free(pairs, batch)


def test_batch_membership_rules():
    pairs = _pairs(MEMBERS[:2])
    batch = F.fciqmc_batch_create()
    (_, r0, s0), (_, r1, s1) = pairs
    F.fciqmc_batch_add(batch, r0)
    F.fciqmc_batch_add(batch, r1)
    with pytest.raises(F.FciqmcError) as e:
        F.fciqmc_step(r0, 1)
    assert e.value.code == F.ESTATE
    other = F.fciqmc_batch_create()
    with pytest.raises(F.FciqmcError) as e:
        F.fciqmc_batch_add(other, r0)
    assert e.value.code == F.EINVAL
    with pytest.raises(F.FciqmcError):
        F.fciqmc_batch_remove(other, r0)
    F.fciqmc_batch_free(other)
    F.fciqmc_batch_step(batch, 30)
    # leave the batch: the run continues alone on its own stream
    F.fciqmc_batch_remove(batch, r0)
    assert F.fciqmc_batch_size(batch) == 1
    a = F.fciqmc_step(r0, 30)
    b = F.fciqmc_step(s0, 60)
    assert_same_gpu_stats(a[-1], b[-1])
    assert_same_gpu_walkers(r0, s0)
    # energies stay available for members
    F.fciqmc_energy(r1)
    # an empty batch steps as a no-op; a freed member leaves its batch
    F.fciqmc_free_run(r1)
    assert F.fciqmc_batch_size(batch) == 0
    F.fciqmc_batch_step(batch, 2)
    F.fciqmc_batch_free(batch)
    for sysd, rb, rs in pairs:
        F.fciqmc_free_run(rb)
        F.fciqmc_free_run(rs)
        F.fciqmc_free_system(sysd)


def test_batch_real_mode_matches_solo():
    """Real coefficients (two-word layout, PCHB): amplitudes summed in another
    order agree to rounding; the determinant sets agree."""
    s = inputs.synthetic_molecule(10, 4, 4, seed=2)
    kw = dict(tau=0.02, target=1e9, mode="real", seed=4, gen="pchb", det_words=2)
    sysd, rb = make_gpu_run(s, **kw)
    _, rs = make_gpu_run(s, sysd=sysd, **kw)
    ra, rb_ = ref_of(s)
    a, b, v = inputs.random_walker_state(10, 4, 4, 400, seed=5, max_pop=10, integer=False,
                                         include=(ra, rb_))
    F.fciqmc_set_walkers(rb, a, b, v)
    F.fciqmc_set_walkers(rs, a, b, v)
    other = _pairs(MEMBERS[:1])
    batch = F.fciqmc_batch_create()
    F.fciqmc_batch_add(batch, other[0][1])
    F.fciqmc_batch_add(batch, rb)
    g = F.fciqmc_batch_step(batch, 1)[0][1]
    o = F.fciqmc_step(rs, 1)[0]
    assert g["ndets"] == o["ndets"] and g["spawns"] == o["spawns"]
    assert abs(g["nw"] - o["nw"]) <= 1e-12 * o["nw"]
    assert_same_gpu_walkers(rb, rs, exact=False, rtol=1e-12)
    F.fciqmc_batch_free(batch)
    F.fciqmc_free_run(rb)
    F.fciqmc_free_run(rs)
    F.fciqmc_free_system(sysd)
    _free(other)
