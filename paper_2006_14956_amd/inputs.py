"""Seeded synthetic inputs for the FCIQMC step.

This module only *generates input data* (integrals, lattices, reference
determinants).  It holds none of the method's arithmetic: no matrix elements,
no excitation generation, no walker dynamics.  Both the HIP path and the CPU
oracle consume its output, which is why it lives on its own.

The paper feeds the method an integral file (one- and two-electron integrals
h_pq and (pq|rs), Sec. "Interfaces" and the transcorrelated section where the
integrals are named) and supports real-space Hubbard lattices (Introduction).
None of the paper's molecular integrals are available, so the molecules here
are synthetic stand-ins with the structure of an ab initio Hamiltonian:

* h is symmetric, its diagonal is N uniform draws in [-2, 1] sorted ascending,
  its off-diagonal entries are N(0, 0.05) (standard deviation 0.05);
* (pq|rs) = sum_k L^k_pq L^k_rs with L^k symmetric and L ~ N(0, 0.1), so the
  two-electron tensor has the full 8-fold permutational symmetry and is a
  positive semi-definite Coulomb-like kernel;
* optionally |L^k_pq| is damped by exp(-|p - q| / damping) (a locality proxy).

Two-electron integrals are passed around 8-fold packed in chemists' notation:
P = p(p+1)/2 + q for p >= q, and (pq|rs) sits at P(P+1)/2 + Q with P >= Q.
"""
from __future__ import annotations

import dataclasses

import numpy as np


def pair_index(p: int, q: int) -> int:
    """Triangular index of an unordered pair (p, q)."""
    if p < q:
        p, q = q, p
    return p * (p + 1) // 2 + q


def eri_packed_len(n_orb: int) -> int:
    m = n_orb * (n_orb + 1) // 2
    return m * (m + 1) // 2


def pack_eri(eri4: np.ndarray) -> np.ndarray:
    """Pack a full (N,N,N,N) chemists'-notation tensor with 8-fold symmetry."""
    n = eri4.shape[0]
    out = np.zeros(eri_packed_len(n), dtype=np.float64)
    for p in range(n):
        for q in range(p + 1):
            pq = p * (p + 1) // 2 + q
            for r in range(n):
                for s in range(r + 1):
                    rs = r * (r + 1) // 2 + s
                    if rs > pq:
                        continue
                    out[pq * (pq + 1) // 2 + rs] = eri4[p, q, r, s]
    return out


def unpack_eri(packed: np.ndarray, n: int) -> np.ndarray:
    """Expand an 8-fold packed tensor to the full (N,N,N,N) array (values copied, no arithmetic)."""
    m = n * (n + 1) // 2
    idx = np.zeros((n, n), dtype=np.int64)
    for p in range(n):
        for q in range(n):
            idx[p, q] = pair_index(p, q)
    P = idx[:, :, None, None]
    Q = idx[None, None, :, :]
    hi = np.maximum(P, Q)
    lo = np.minimum(P, Q)
    flat = hi * (hi + 1) // 2 + lo
    assert packed.shape[0] == m * (m + 1) // 2
    return packed[flat]


@dataclasses.dataclass
class System:
    """Integrals plus electron counts: exactly what the integral-loading call takes."""
    name: str
    n_orb: int
    n_alpha: int
    n_beta: int
    e_core: float
    h1: np.ndarray          # (N, N) float64, symmetric
    eri: np.ndarray         # packed, float64
    ref_alpha: int = 0      # reference determinant as spatial-orbital masks (0 = aufbau)
    ref_beta: int = 0

    @property
    def n_elec(self) -> int:
        return self.n_alpha + self.n_beta


def synthetic_molecule(n_orb: int, n_alpha: int, n_beta: int, seed: int,
                       rank: int = 16, damping: float | None = None,
                       h_offdiag_sd: float = 0.05, l_sd: float = 0.1,
                       name: str | None = None) -> System:
    """Seeded synthetic molecular integrals (see module docstring for the recipe)."""
    rng = np.random.default_rng(seed)
    eps = np.sort(rng.uniform(-2.0, 1.0, size=n_orb))
    off = rng.normal(0.0, h_offdiag_sd, size=(n_orb, n_orb))
    up = np.triu(off, 1)
    h1 = up + up.T + np.diag(eps)
    L = rng.normal(0.0, l_sd, size=(rank, n_orb, n_orb))
    L = np.triu(L) + np.transpose(np.triu(L, 1), (0, 2, 1))
    if damping is not None:
        p = np.arange(n_orb)
        L = L * np.exp(-np.abs(p[:, None] - p[None, :]) / damping)[None]
    eri4 = np.einsum("kpq,krs->pqrs", L, L)
    # enforce exact 8-fold symmetry bit-for-bit before packing
    eri4 = 0.5 * (eri4 + eri4.transpose(2, 3, 0, 1))
    return System(name=name or f"mol{n_orb}o{n_alpha + n_beta}e_s{seed}", n_orb=n_orb,
                  n_alpha=n_alpha, n_beta=n_beta, e_core=0.0, h1=h1, eri=pack_eri(eri4))


def lattice_bonds(lx: int, ly: int, periodic: bool = True) -> list[tuple[int, int]]:
    """Nearest-neighbour bonds of an lx-by-ly square lattice, site = x + lx*y.

    Bonds are a set of unordered site pairs: on a periodic side of length 2 the
    +1 and -1 neighbours coincide and give one bond, not two.
    """
    bonds = set()
    for y in range(ly):
        for x in range(lx):
            s = x + lx * y
            for dx, dy in ((1, 0), (0, 1)):
                xx, yy = x + dx, y + dy
                if xx >= lx:
                    if not periodic or lx < 2:
                        continue
                    xx -= lx
                if yy >= ly:
                    if not periodic or ly < 2:
                        continue
                    yy -= ly
                t = xx + lx * yy
                if t != s:
                    bonds.add((min(s, t), max(s, t)))
    return sorted(bonds)


def hubbard(lx: int, ly: int, t: float, u: float, n_alpha: int, n_beta: int,
            periodic: bool = True, neel: bool = True, name: str | None = None) -> System:
    """Real-space Hubbard model as integrals: h_pq = -t on bonds, (pp|pp) = U."""
    n = lx * ly
    h1 = np.zeros((n, n))
    for p, q in lattice_bonds(lx, ly, periodic):
        h1[p, q] = -t
        h1[q, p] = -t
    eri = np.zeros(eri_packed_len(n))
    for p in range(n):
        pp = pair_index(p, p)
        eri[pp * (pp + 1) // 2 + pp] = u
    ref_a = ref_b = 0
    if neel:
        even = [x + lx * y for y in range(ly) for x in range(lx) if (x + y) % 2 == 0]
        odd = [x + lx * y for y in range(ly) for x in range(lx) if (x + y) % 2 == 1]
        if n_alpha > len(even) or n_beta > len(odd):
            raise ValueError("Neel reference needs n_alpha <= #even sites and n_beta <= #odd sites")
        for s in even[:n_alpha]:
            ref_a |= 1 << s
        for s in odd[:n_beta]:
            ref_b |= 1 << s
    return System(name=name or f"hubbard{lx}x{ly}_U{u}", n_orb=n, n_alpha=n_alpha,
                  n_beta=n_beta, e_core=0.0, h1=h1, eri=eri, ref_alpha=ref_a, ref_beta=ref_b)


def hubbard_chain(length: int, t: float, u: float, n_alpha: int, n_beta: int,
                  periodic: bool = True) -> System:
    """1D Hubbard ring/chain (a 1-by-L lattice); the Neel reference alternates spins."""
    s = hubbard(length, 1, t, u, n_alpha, n_beta, periodic=periodic, neel=True,
                name=f"hubbard_chain{length}_U{u}")
    return s


# --- the named workloads --------------------------------------------------------------

def molecule_8o8e(seed: int = 0) -> System:
    """8 electrons in 8 spatial orbitals, Sz = 0 (4900 determinants), rank-16 kernel."""
    return synthetic_molecule(8, 4, 4, seed=seed, rank=16, name="mol_8o8e")


def hubbard_4x4(u: float = 4.0, t: float = 1.0) -> System:
    """4x4 periodic real-space Hubbard model, 8 up + 8 down electrons, Neel reference."""
    return hubbard(4, 4, t, u, 8, 8, periodic=True, neel=True, name=f"hubbard_4x4_U{u:g}")


def molecule_40o26e(seed: int = 0) -> System:
    """26 electrons in 40 spatial orbitals (80 spin orbitals), rank 40, |L| damped by exp(-|p-q|/8)."""
    return synthetic_molecule(40, 13, 13, seed=seed, rank=40, damping=8.0, name="mol_40o26e")


def batched_molecules(count: int = 64, lo: int = 8, hi: int = 24) -> list[tuple[System, float]]:
    """Independent molecules: orbitals uniform in [lo, hi], electrons = orbitals rounded
    down to even (half filling, Sz = 0), walker target log-uniform in [1e4, 1e6].

    Returns (system, walker_target) pairs; instance i uses integral seed i.
    """
    out = []
    for i in range(count):
        r = np.random.default_rng(1000 + i)
        n_orb = int(r.integers(lo, hi + 1))
        n_el = 2 * (n_orb // 2)
        target = float(10.0 ** r.uniform(4.0, 6.0))
        out.append((synthetic_molecule(n_orb, n_el // 2, n_el // 2, seed=i, rank=16,
                                       name=f"batch{i}_{n_orb}o{n_el}e"), target))
    return out


def random_walker_state(n_orb: int, n_alpha: int, n_beta: int, n_dets: int, seed: int,
                        max_pop: int = 20, integer: bool = True,
                        include: tuple[int, int] | None = None):
    """A seeded random sparse walker state: distinct determinants with signed populations.

    Returns (alpha_masks, beta_masks, values) as numpy arrays (uint64, uint64, float64).
    """
    rng = np.random.default_rng(seed)
    seen = set()
    dets = []
    if include is not None:
        seen.add(include)
        dets.append(include)
    while len(dets) < n_dets:
        a = rng.choice(n_orb, size=n_alpha, replace=False)
        b = rng.choice(n_orb, size=n_beta, replace=False)
        am = 0
        bm = 0
        for x in a:
            am |= 1 << int(x)
        for x in b:
            bm |= 1 << int(x)
        if (am, bm) in seen:
            continue
        seen.add((am, bm))
        dets.append((am, bm))
    if integer:
        vals = rng.integers(1, max_pop + 1, size=len(dets)).astype(np.float64)
    else:
        vals = rng.uniform(0.05, float(max_pop), size=len(dets))
    vals *= rng.choice([-1.0, 1.0], size=len(dets))
    am = np.array([d[0] for d in dets], dtype=np.uint64)
    bm = np.array([d[1] for d in dets], dtype=np.uint64)
    return am, bm, vals
