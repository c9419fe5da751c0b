"""GPU parity at the edges of the supported inputs: the largest orbital
counts of both determinant layouts, spin-polarised systems (no beta
electrons), and a population that dies out."""
import numpy as np
import pytest

from paper_2006_14956_amd import fciqmc as F
from paper_2006_14956_amd import inputs
from tests.gpu_helpers import assert_same_stats, assert_same_walkers, make_pair, ref_of

pytestmark = pytest.mark.gpu


def _steps(run, orun, n, block):
    for _ in range(n // block):
        g = F.fciqmc_step(run, block)
        o = orun.step(block)
        for gg, oo in zip(g, o):
            assert_same_stats(gg, oo)
        assert_same_walkers(run, orun)
    return g


@pytest.mark.parametrize("n_orb,words,gen", [(63, 2, "uniform"), (63, 2, "pe"), (63, 2, "cs"), (63, 2, "pchb"),
                                             (32, 1, "uniform"), (32, 1, "pchb"), (45, 2, "cs"), (46, 2, "cs")])
def test_largest_orbital_counts(n_orb, words, gen):
    """63 orbitals (every bit but the top of both words) and 32 orbitals (the
    full one-word layout): a random population, one step and five more.  45
    and 46 orbitals bracket the largest system whose Cauchy-Schwarz tables
    the spawn kernel keeps in LDS; at 63 orbitals the heat-bath tables have
    their most columns (3969 per opposite-spin row), the widest alias field
    of a packed entry."""
    s = inputs.synthetic_molecule(n_orb, 3, 2, seed=31, rank=6)
    sysd, run, orun = make_pair(s, tau=0.002, target=1e9, gen=gen, det_words=words, seed=5, n_a=2.0)
    ra, rb = ref_of(s)
    a, b, v = inputs.random_walker_state(n_orb, 3, 2, 200, seed=4, max_pop=20, include=(ra, rb))
    # a determinant that uses the highest orbital of each spin
    top = (1 << (n_orb - 1)) | 3, (1 << (n_orb - 1)) | 1
    if top not in set(zip(a.tolist(), b.tolist())):
        a = np.append(a, np.uint64(top[0]))
        b = np.append(b, np.uint64(top[1]))
        v = np.append(v, 7.0)
    F.fciqmc_set_walkers(run, a, b, v)
    orun.set_walkers(a, b, v)
    _steps(run, orun, 1, 1)
    _steps(run, orun, 5, 5)
    F.fciqmc_free_run(run)
    F.fciqmc_free_system(sysd)


@pytest.mark.parametrize("gen", ["uniform", "pchb", "cs"])
def test_spin_polarised(gen):
    """Four alpha electrons and no beta electron in 9 orbitals: only
    equal-spin excitations exist; 200 steps from the reference."""
    s = inputs.synthetic_molecule(9, 4, 0, seed=13)
    sysd, run, orun = make_pair(s, tau=0.01, target=2e3, gen=gen, seed=3)
    g = _steps(run, orun, 200, 50)
    assert g[-1]["nw"] > 0
    F.fciqmc_free_run(run)
    F.fciqmc_free_system(sysd)


def test_population_dies_out():
    """A shift of -1/dtau makes every death factor nearly zero, which drains
    a small population to zero walkers; steps on the empty population keep
    agreeing (nothing to spawn)."""
    s = inputs.molecule_8o8e()
    sysd, run, orun = make_pair(s, tau=0.001, target=1e9, seed=7)
    ra, rb = ref_of(s)
    a, b, v = inputs.random_walker_state(8, 4, 4, 30, seed=2, max_pop=3, include=(ra, rb))
    F.fciqmc_set_walkers(run, a, b, v)
    orun.set_walkers(a, b, v)
    F.fciqmc_set_checkpoint(run, 0, -1000.0, 0, 0, float(np.abs(v).sum()))
    orun.set_state(0, -1000.0, 0, 0, float(np.abs(v).sum()))
    g = _steps(run, orun, 60, 20)
    assert g[-1]["nw"] == 0 and g[-1]["ndets"] == 0 and g[-1]["attempts"] == 0
    F.fciqmc_free_run(run)
    F.fciqmc_free_system(sysd)
