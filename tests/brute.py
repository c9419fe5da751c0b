"""Independent checkers for the oracle (test helpers).

Second-quantised Hamiltonian applied operator by operator to occupation
bit strings, and the basis enumeration.  Written from the definition
H = sum_pq h_pq a+_p a_q + 1/2 sum_pqrs <pq|rs> a+_p a+_q a_s a_r with
<pq|rs> = (pr|qs) delta(spin p, spin r) delta(spin q, spin s), shares
nothing with the oracle's Slater-Condon code.
"""
from itertools import combinations

import numpy as np


def basis(n_orb, n_alpha, n_beta):
    """All determinants as (alpha_mask, beta_mask), alpha-major order."""
    out = []
    for a in combinations(range(n_orb), n_alpha):
        am = sum(1 << p for p in a)
        for b in combinations(range(n_orb), n_beta):
            bm = sum(1 << p for p in b)
            out.append((am, bm))
    return out


def _to_so(am, bm, n):
    return am | (bm << n)


def _from_so(x, n):
    return x & ((1 << n) - 1), x >> n


def _annihilate(x, p):
    if not (x >> p) & 1:
        return None, 0
    sign = -1 if bin(x & ((1 << p) - 1)).count("1") % 2 else 1
    return x & ~(1 << p), sign


def _create(x, p):
    if (x >> p) & 1:
        return None, 0
    sign = -1 if bin(x & ((1 << p) - 1)).count("1") % 2 else 1
    return x | (1 << p), sign


def hamiltonian(n_orb, n_alpha, n_beta, h1, eri4):
    """Dense H over basis(), built by applying every operator string."""
    dets = basis(n_orb, n_alpha, n_beta)
    index = {d: i for i, d in enumerate(dets)}
    D = len(dets)
    H = np.zeros((D, D))
    n2 = 2 * n_orb
    spin = [0] * n_orb + [1] * n_orb
    orb = list(range(n_orb)) * 2
    for col, (am, bm) in enumerate(dets):
        x = _to_so(am, bm, n_orb)
        occ = [p for p in range(n2) if (x >> p) & 1]
        # one-body
        for q in occ:
            y, s1 = _annihilate(x, q)
            for p in range(n2):
                if spin[p] != spin[q]:
                    continue
                z, s2 = _create(y, p)
                if z is None:
                    continue
                row = index[_from_so(z, n_orb)]
                H[row, col] += s1 * s2 * h1[orb[p], orb[q]]
        # two-body: 1/2 <pq|rs> a+_p a+_q a_s a_r
        for r in occ:
            y1, s1 = _annihilate(x, r)
            for s in occ:
                if s == r:
                    continue
                y2, s2 = _annihilate(y1, s)
                for q in range(n2):
                    if spin[q] != spin[s]:
                        continue
                    y3, s3 = _create(y2, q)
                    if y3 is None:
                        continue
                    for p in range(n2):
                        if spin[p] != spin[r]:
                            continue
                        y4, s4 = _create(y3, p)
                        if y4 is None:
                            continue
                        v = eri4[orb[p], orb[r], orb[q], orb[s]]
                        if v == 0.0:
                            continue
                        row = index[_from_so(y4, n_orb)]
                        H[row, col] += 0.5 * s1 * s2 * s3 * s4 * v
    return dets, H


def oracle_dense_h(osys, dets):
    """Dense H from the oracle's pairwise matrix elements."""
    D = len(dets)
    H = np.zeros((D, D))
    for i, (a1, b1) in enumerate(dets):
        for j, (a2, b2) in enumerate(dets):
            if i == j:
                H[i, i] = osys.hdiag(a1, b1)
            else:
                x = bin(a1 ^ a2).count("1") + bin(b1 ^ b2).count("1")
                if x <= 4:
                    H[j, i] = osys.hij(a1, b1, a2, b2)
    return H


def blocking(series):
    """Flyvbjerg-Petersen blocking: (mean, list of (block_len, error, error_of_error))."""
    x = np.asarray(series, dtype=np.float64)
    mean = x.mean()
    out = []
    blen = 1
    while len(x) >= 2:
        n = len(x)
        var = x.var(ddof=0)
        err = np.sqrt(var / (n - 1))
        out.append((blen, err, err / np.sqrt(2.0 * (n - 1))))
        m = n // 2
        x = 0.5 * (x[0:2 * m:2] + x[1:2 * m:2])
        blen *= 2
    return mean, out


def blocked_error(series):
    """Plateau estimate: the first block level whose error is within the
    error-of-error of every larger level (Flyvbjerg-Petersen criterion)."""
    mean, levels = blocking(series)
    for i, (bl, err, derr) in enumerate(levels):
        rest = levels[i + 1:]
        if len(levels) - i < 4:
            break
        if all(abs(e - err) <= 2.0 * (derr + de) for _, e, de in rest[:3]):
            return mean, err
    return mean, max(e for _, e, _ in levels[: max(1, len(levels) - 3)])


def rdm2(n_orb, dets, ca, cb):
    """Gamma_{kl,mn} = sum_{i,j} ca_i cb_j <D_i| a+_k a+_l a_n a_m |D_j> for
    spin orbitals k < l, m < n (alpha 0..N-1, then beta), by applying the
    four operators to every ket, right to left.  Rows and columns run over
    the pairs in lexicographic order."""
    n2 = 2 * n_orb
    pairs = [(k, l) for k in range(n2) for l in range(k + 1, n2)]
    pidx = {p: i for i, p in enumerate(pairs)}
    index = {d: i for i, d in enumerate(dets)}
    M = len(pairs)
    G = np.zeros((M, M))
    for j, (am, bm) in enumerate(dets):
        if cb[j] == 0.0:
            continue
        x = _to_so(am, bm, n_orb)
        for (m, n) in pairs:
            y1, s1 = _annihilate(x, m)
            if y1 is None:
                continue
            y2, s2 = _annihilate(y1, n)
            if y2 is None:
                continue
            for (k, l) in pairs:
                y3, s3 = _create(y2, l)
                if y3 is None:
                    continue
                y4, s4 = _create(y3, k)
                if y4 is None:
                    continue
                i = index.get(_from_so(y4, n_orb))
                if i is None or ca[i] == 0.0:
                    continue
                G[pidx[(k, l)], pidx[(m, n)]] += s1 * s2 * s3 * s4 * ca[i] * cb[j]
    return G
