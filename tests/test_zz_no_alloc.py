"""The allocation-free matrix-element entry point against the allocating
one: the same values bit for bit on two calls in a row (the second
smaller, so stale staging would show), through the C ABI, plus its size
limit."""
import numpy as np
import pytest

from paper_2006_14956_amd import fciqmc as F
from paper_2006_14956_amd import inputs

pytestmark = pytest.mark.gpu


def _pairs(s, n, seed):
    """n (D_i, D_j) pairs: a quarter diagonal, the rest D_j a random single or
    double excitation of D_i or an unrelated determinant."""
    rng = np.random.default_rng(seed)
    a, b, _ = inputs.random_walker_state(s.n_orb, s.n_alpha, s.n_beta, min(n, 3000), seed=seed)
    pick = rng.integers(len(a), size=n)
    di = np.stack([a[pick], b[pick]], axis=1).astype(np.uint64)
    dj = di.copy()
    N = s.n_orb
    for k in range(n):
        kind = k % 4
        if kind == 0:
            continue
        if kind == 3:
            j = rng.integers(n)
            dj[k] = di[j]
            continue
        words = [int(di[k, 0]), int(di[k, 1])]
        for _ in range(kind):  # one or two electrons moved within their spin
            sp = int(rng.integers(2))
            occ = [p for p in range(N) if (words[sp] >> p) & 1]
            vir = [p for p in range(N) if not (words[sp] >> p) & 1]
            if not occ or not vir:
                continue
            words[sp] ^= (1 << int(rng.choice(occ))) | (1 << int(rng.choice(vir)))
        dj[k] = words
    return di, dj


@pytest.mark.parametrize("system", ["mol8", "mol40"])
def test_noalloc_matches_allocating_entry_point(system):
    s = inputs.molecule_8o8e() if system == "mol8" else inputs.molecule_40o26e()
    sysd = F.fciqmc_load_integrals(s.n_orb, s.n_alpha, s.n_beta, s.e_core, s.h1, s.eri)
    for n, seed in ((60000, 1), (777, 2)):
        di, dj = _pairs(s, n, seed)
        want = F.fciqmc_matrix_elements(sysd, di, dj)
        got = F.fciqmc_matrix_elements_noalloc(sysd, di, dj)
        assert got.shape == want.shape == (n,)
        assert np.array_equal(got, want), int(np.argmax(got != want))
        assert np.count_nonzero(want) > n // 3
    F.fciqmc_free_system(sysd)


def test_noalloc_size_limit():
    s = inputs.molecule_8o8e()
    sysd = F.fciqmc_load_integrals(s.n_orb, s.n_alpha, s.n_beta, s.e_core, s.h1, s.eri)
    di, dj = _pairs(s, 65537, 3)
    with pytest.raises(F.FciqmcError) as e:
        F.fciqmc_matrix_elements_noalloc(sysd, di, dj)
    assert e.value.code == F.EINVAL
    # the limit itself is accepted, and the call after a refused one is right
    got = F.fciqmc_matrix_elements_noalloc(sysd, di[:65536], dj[:65536])
    assert np.array_equal(got, F.fciqmc_matrix_elements(sysd, di[:65536], dj[:65536]))
    assert len(F.fciqmc_matrix_elements_noalloc(sysd, di[:0], dj[:0])) == 0
    F.fciqmc_free_system(sysd)
