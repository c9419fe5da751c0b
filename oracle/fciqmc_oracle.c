/*
 * Plain, slow CPU oracle for one FCIQMC imaginary-time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code with the HIP path.
 *
 * Every routine follows the paper (Guther et al., "NECI: N-Electron
 * Configuration Interaction with an emphasis on state-of-the-art stochastic
 * methods", J. Chem. Phys. 2020) or a textbook definition it relies on, and
 * says which.  Readings of passages that the paper leaves open are marked
 * "Reading:".  Floating point is IEEE binary64 evaluated one operation at a
 * time (built with -ffp-contract=off, no fast-math): every `x = y op z` below
 * is one rounding, in the order written.
 *
 * Determinants.  A determinant is an occupation bit string over 2N spin
 * orbitals (Appendix A, "Stochastic excitation generation and p_gen").  Internally the
 * oracle keeps it as two spatial-orbital masks (alpha, beta).  Canonical
 * spin-orbital order (Reading: the paper fixes no order) is all alpha
 * orbitals 0..N-1 first, then all beta orbitals (canonical index N+p).
 * Two storage layouts are used to key the random numbers:
 *   1 word  (N <= 32): alpha in bits 0..31, beta in bits 32..63;
 *   2 words (N <= 64): word 0 = alpha, word 1 = beta.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,        */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of two  */
/* 32x32->64 multiplies with a Weyl-sequence key schedule.  The paper uses a */
/* sequential Mersenne twister (dSFMT, Sec. I); Reading: a counter-based     */
/* stream keyed by the walker's identity replaces it so that the result does */
/* not depend on how walkers are distributed over threads.                   */
/* ------------------------------------------------------------------------- */
#define PHILOX_M0 0xD2511F53U
#define PHILOX_M1 0xCD9E8D57U
#define PHILOX_W0 0x9E3779B9U
#define PHILOX_W1 0xBB67AE85U

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* splitmix64 finaliser (Steele, Lea, Flood, OOPSLA'14), a bijection of 64-bit */
/* words; it hashes the stream identity into Philox keys and counters below.  */
static uint64_t splitmix64_fin(uint64_t x)
{
    x ^= x >> 30; x *= 0xBF58476D1CE4E5B9ULL;
    x ^= x >> 27; x *= 0x94D049BB133111EBULL;
    x ^= x >> 31;
    return x;
}

/* Discrete choice in [0, m): floor(x * m / 2^64). */
static uint64_t pick(uint64_t x, uint64_t m)
{
    return (uint64_t)(((u128)x * (u128)m) >> 64);
}

/* Uniform double in [0, 1) with 53 random bits. */
static double unif(uint64_t x)
{
    return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

enum { PURPOSE_SPAWN = 0, PURPOSE_SPAWN2 = 1, PURPOSE_DEATH = 2, PURPOSE_ANN = 4 };

/* ------------------------------------------------------------------------- */
/* System: integrals and derived tables.                                      */
/* ------------------------------------------------------------------------- */
typedef struct { uint64_t a, b; } det_t;

typedef struct {
    int N, na, nb, words;
    double e_core;
    double *h;      /* N*N, h[p*N+q] */
    double *eri4;   /* N^4 chemists' (pq|rs) at ((p*N+q)*N+r)*N+s */
    int *deg;       /* lattice degree per site */
    int *nbr;       /* N*N: ascending neighbour list of each site */
    /* pre-computed heat-bath tables (Appendix A.3) */
    double *hb_w_same;   /* [pair I<J][pair A<B] weights over spatial indices */
    double *hb_w_opp;    /* [I*N+J][A*N+B] weights */
    double *hb_sum_same; /* per (i<j) */
    double *hb_sum_opp;  /* per (I,J) */
    double *hb_p_same, *hb_p_opp; /* alias keep-probabilities */
    int *hb_a_same, *hb_a_opp;    /* alias columns */
} orc_sys;

static double eri(const orc_sys *s, int p, int q, int r, int t)
{
    int N = s->N;
    return s->eri4[((size_t)(p * N + q) * N + r) * N + t];
}

static int tri(int p, int q) { return p >= q ? p * (p + 1) / 2 + q : q * (q + 1) / 2 + p; }

/* Load integrals: h (N*N) and the 8-fold packed (pq|rs). The full tensor is
 * filled by copying packed values to every permutation (no arithmetic). */
orc_sys *orc_sys_create(int N, int na, int nb, double e_core, const double *h,
                        const double *eri_packed)
{
    orc_sys *s = (orc_sys *)calloc(1, sizeof(orc_sys));
    s->N = N; s->na = na; s->nb = nb; s->e_core = e_core;
    s->words = (N <= 32) ? 1 : 2;
    s->h = (double *)malloc(sizeof(double) * N * N);
    memcpy(s->h, h, sizeof(double) * N * N);
    s->eri4 = (double *)malloc(sizeof(double) * (size_t)N * N * N * N);
    for (int p = 0; p < N; ++p)
        for (int q = 0; q < N; ++q)
            for (int r = 0; r < N; ++r)
                for (int t = 0; t < N; ++t) {
                    int P = tri(p, q), Q = tri(r, t);
                    int PQ = tri(P, Q);
                    s->eri4[((size_t)(p * N + q) * N + r) * N + t] = eri_packed[PQ];
                }
    /* lattice neighbours: the distinct q != p with h_pq != 0, ascending */
    s->deg = (int *)calloc(N, sizeof(int));
    s->nbr = (int *)calloc((size_t)N * N, sizeof(int));
    for (int p = 0; p < N; ++p)
        for (int q = 0; q < N; ++q)
            if (q != p && h[p * N + q] != 0.0)
                s->nbr[p * N + s->deg[p]++] = q;
    return s;
}

void orc_sys_set_words(orc_sys *s, int words) { s->words = words; }

void orc_sys_free(orc_sys *s)
{
    if (!s) return;
    free(s->h); free(s->eri4); free(s->deg); free(s->nbr);
    free(s->hb_w_same); free(s->hb_w_opp); free(s->hb_sum_same); free(s->hb_sum_opp);
    free(s->hb_p_same); free(s->hb_p_opp); free(s->hb_a_same); free(s->hb_a_opp);
    free(s);
}

/* ------------------------------------------------------------------------- */
/* Determinant helpers, by explicit loops over spin orbitals.                */
/* ------------------------------------------------------------------------- */
static int so_spin(const orc_sys *s, int so) { return so >= s->N; }        /* 0 alpha, 1 beta */
static int so_orb(const orc_sys *s, int so) { return so >= s->N ? so - s->N : so; }

static int det_occ(const orc_sys *s, det_t d, int so)
{
    int p = so_orb(s, so);
    return so_spin(s, so) ? (int)((d.b >> p) & 1) : (int)((d.a >> p) & 1);
}

static void det_set(const orc_sys *s, det_t *d, int so, int v)
{
    int p = so_orb(s, so);
    uint64_t *w = so_spin(s, so) ? &d->b : &d->a;
    if (v) *w |= (1ULL << p); else *w &= ~(1ULL << p);
}

/* Occupied spin orbitals in canonical order. */
static int det_occ_list(const orc_sys *s, det_t d, int *occ)
{
    int n = 0;
    for (int so = 0; so < 2 * s->N; ++so)
        if (det_occ(s, d, so)) occ[n++] = so;
    return n;
}

/* Number of occupied spin orbitals with canonical index below `so`. */
static int det_below(const orc_sys *s, det_t d, int so)
{
    int c = 0;
    for (int x = 0; x < so; ++x) c += det_occ(s, d, x);
    return c;
}

/* Second-quantised operators applied to a determinant, right to left: each
 * contributes (-1)^(occupied orbitals below it in the current string). */
static int op_annihilate(const orc_sys *s, det_t *d, int so)
{
    int par = det_below(s, *d, so) & 1;
    det_set(s, d, so, 0);
    return par;
}

static int op_create(const orc_sys *s, det_t *d, int so)
{
    int par = det_below(s, *d, so) & 1;
    det_set(s, d, so, 1);
    return par;
}

static void layout_words(const orc_sys *s, det_t d, uint64_t *c0, uint64_t *c1)
{
    if (s->words == 1) { *c0 = d.a | (d.b << 32); *c1 = 0; }
    else { *c0 = d.a; *c1 = d.b; }
}

static det_t from_layout(const orc_sys *s, uint64_t w0, uint64_t w1)
{
    det_t d;
    if (s->words == 1) { d.a = w0 & 0xFFFFFFFFULL; d.b = w0 >> 32; }
    else { d.a = w0; d.b = w1; }
    return d;
}

static int det_cmp(det_t x, det_t y)
{
    if (x.a != y.a) return x.a < y.a ? -1 : 1;
    if (x.b != y.b) return x.b < y.b ? -1 : 1;
    return 0;
}

static int det_eq(det_t x, det_t y) { return x.a == y.a && x.b == y.b; }

/* ------------------------------------------------------------------------- */
/* Slater-Condon matrix elements.  The paper gives the double-excitation     */
/* element <ij||ab> = <ij|ab> - <ij|ba> (Appendix, uniform excitation        */
/* generation) and notes that the exchange part vanishes for opposite spins  */
/* (Appendix A.2, Cauchy-Schwarz doubles).  The remaining rules are the textbook */
/* Slater-Condon rules for H = sum h_pq a+_p a_q + 1/2 sum <pq|rs>           */
/* a+_p a+_q a_s a_r with <pq|rs> = (pr|qs) d(s_p,s_r) d(s_q,s_s).           */
/* ------------------------------------------------------------------------- */

/* Diagonal element: sum_p h_pp + sum_{p<q} [(pp|qq) - d(s_p,s_q)(pq|qp)]. */
double orc_hdiag_det(const orc_sys *s, det_t d)
{
    int occ[128];
    int n = det_occ_list(s, d, occ);
    double acc = 0.0;
    for (int x = 0; x < n; ++x) {
        int p = so_orb(s, occ[x]);
        acc = acc + s->h[p * s->N + p];
    }
    for (int x = 0; x < n; ++x)
        for (int y = x + 1; y < n; ++y) {
            int p = so_orb(s, occ[x]), q = so_orb(s, occ[y]);
            if (so_spin(s, occ[x]) != so_spin(s, occ[y])) {
                acc = acc + eri(s, p, p, q, q);
            } else {
                double v = eri(s, p, p, q, q) - eri(s, p, q, q, p);
                acc = acc + v;
            }
        }
    return acc;
}

/* <D_j|H|D_i> for D_j = sgn a+_a a_i D_i (same spin), summing over the
 * electrons of D_i other than i in canonical order. */
static double hsingle(const orc_sys *s, det_t d, int i, int a)
{
    int occ[128];
    int n = det_occ_list(s, d, occ);
    int pi = so_orb(s, i), pa = so_orb(s, a), sig = so_spin(s, i);
    double v = s->h[pi * s->N + pa];
    for (int x = 0; x < n; ++x) {
        int k = occ[x];
        if (k == i) continue;
        int pk = so_orb(s, k);
        if (so_spin(s, k) != sig) {
            v = v + eri(s, pi, pa, pk, pk);
        } else {
            double t = eri(s, pi, pa, pk, pk) - eri(s, pi, pk, pk, pa);
            v = v + t;
        }
    }
    det_t t = d;
    int par = op_annihilate(s, &t, i);
    par ^= op_create(s, &t, a);
    return par ? -v : v;
}

/* <D_j|H|D_i> for D_j = sgn a+_a a+_b a_j a_i D_i, i<j and a<b canonical.
 * The coefficient of that operator string in H is <ab||ij>:
 * (ai|bj) d(s_a,s_i) d(s_b,s_j) - (aj|bi) d(s_a,s_j) d(s_b,s_i). */
static double hdouble(const orc_sys *s, det_t d, int i, int j, int a, int b)
{
    int pi = so_orb(s, i), pj = so_orb(s, j), pa = so_orb(s, a), pb = so_orb(s, b);
    int si = so_spin(s, i), sj = so_spin(s, j), sa = so_spin(s, a), sb = so_spin(s, b);
    double direct = (sa == si && sb == sj) ? eri(s, pa, pi, pb, pj) : 0.0;
    double exch = (sa == sj && sb == si) ? eri(s, pa, pj, pb, pi) : 0.0;
    double v;
    if (si == sj) v = direct - exch;     /* same spin: both terms */
    else v = (sa == si) ? direct : -exch; /* opposite spin: one term survives */
    det_t t = d;
    int par = op_annihilate(s, &t, i);
    par ^= op_annihilate(s, &t, j);
    par ^= op_create(s, &t, b);
    par ^= op_create(s, &t, a);
    return par ? -v : v;
}

/* Generic <D2|H|D1> by excitation level (0, 1, 2; zero beyond). */
double orc_hij_det(const orc_sys *s, det_t d1, det_t d2)
{
    int rem[4], add[4], nr = 0, na = 0;
    for (int so = 0; so < 2 * s->N; ++so) {
        int o1 = det_occ(s, d1, so), o2 = det_occ(s, d2, so);
        if (o1 && !o2) { if (nr < 4) rem[nr] = so; nr++; }
        if (!o1 && o2) { if (na < 4) add[na] = so; na++; }
    }
    if (nr != na) return 0.0;
    if (nr == 0) return orc_hdiag_det(s, d1);
    if (nr == 1) {
        if (so_spin(s, rem[0]) != so_spin(s, add[0])) return 0.0;
        return hsingle(s, d1, rem[0], add[0]);
    }
    if (nr == 2) {
        int sr = so_spin(s, rem[0]) + so_spin(s, rem[1]);
        int sa = so_spin(s, add[0]) + so_spin(s, add[1]);
        if (sr != sa) return 0.0;
        return hdouble(s, d1, rem[0], rem[1], add[0], add[1]);
    }
    return 0.0;
}

/* ------------------------------------------------------------------------- */
/* Excitation generators.  Each returns 1 and fills (target, p_gen, H) or    */
/* returns 0 for a null draw.  p_gen is the exact probability of producing   */
/* the target from this determinant (Sec. II; the spawn is unbiased if       */
/* p_gen > 0 wherever H != 0).                                               */
/* ------------------------------------------------------------------------- */

/* Unoccupied spin orbitals of spin sigma, ascending. */
static int holes_of_spin(const orc_sys *s, det_t d, int sigma, int *out)
{
    int h = 0;
    for (int p = 0; p < s->N; ++p) {
        int so = sigma ? s->N + p : p;
        if (!det_occ(s, d, so)) out[h++] = so;
    }
    return h;
}

/* Count of choices for the uniform generator's second index, given the first. */
uint64_t orc_uniform_count2(const orc_sys *s, det_t d, int single, uint64_t idx1)
{
    int occ[128], hol[64], hb[64];
    int n = det_occ_list(s, d, occ);
    if (single) {
        int sig = so_spin(s, occ[idx1]);
        return (uint64_t)holes_of_spin(s, d, sig, hol);
    }
    int e1 = -1, e2 = -1;
    uint64_t c = 0;
    for (int x = 0; x < n && e1 < 0; ++x)
        for (int y = x + 1; y < n; ++y) {
            if (c == idx1) { e1 = x; e2 = y; break; }
            c++;
        }
    int i = occ[e1], j = occ[e2];
    if (so_spin(s, i) == so_spin(s, j)) {
        uint64_t h = (uint64_t)holes_of_spin(s, d, so_spin(s, i), hol);
        return h * (h - (h > 0)) / 2;
    }
    uint64_t ha = (uint64_t)holes_of_spin(s, d, 0, hol);
    uint64_t hbeta = (uint64_t)holes_of_spin(s, d, 1, hb);
    return ha * hbeta;
}

/* Uniform generator after the random indices have been drawn (Appendix A.1,
 * uniform generation with spin imposed through conditional probabilities):
 *   single: electron idx1 of the n occupied (canonical order), hole idx2 of
 *           the same-spin holes (ascending);
 *           p_gen = p_single / (n * h_sigma);
 *   double: electron pair idx1 of the C(n,2) pairs (lexicographic);
 *           same spin: hole pair idx2 of C(h_sigma,2) same-spin pairs (lexicographic);
 *           opposite:  idx2 = A*h_beta + B picks alpha hole A and beta hole B;
 *           p_gen = (1 - p_single) / (C(n,2) * #hole pairs). */
int orc_uniform_apply(const orc_sys *s, det_t d, int single, uint64_t idx1, uint64_t idx2,
                      double p_single, det_t *tgt, double *pgen)
{
    int occ[128], hol[64], ha[64], hb[64];
    int n = det_occ_list(s, d, occ);
    if (single) {
        int i = occ[idx1];
        int h = holes_of_spin(s, d, so_spin(s, i), hol);
        if (h == 0) return 0;
        int a = hol[idx2];
        det_t t = d; det_set(s, &t, i, 0); det_set(s, &t, a, 1);
        *tgt = t;
        *pgen = p_single / (double)((uint64_t)n * (uint64_t)h);
        return 1;
    }
    uint64_t npair = (uint64_t)n * (uint64_t)(n - 1) / 2;
    int e1 = -1, e2 = -1;
    uint64_t c = 0;
    for (int x = 0; x < n && e1 < 0; ++x)
        for (int y = x + 1; y < n; ++y) {
            if (c == idx1) { e1 = x; e2 = y; break; }
            c++;
        }
    int i = occ[e1], j = occ[e2];
    int a, b;
    uint64_t nh;
    if (so_spin(s, i) == so_spin(s, j)) {
        int h = holes_of_spin(s, d, so_spin(s, i), hol);
        if (h < 2) return 0;
        nh = (uint64_t)h * (uint64_t)(h - 1) / 2;
        int f1 = -1, f2 = -1;
        uint64_t cc = 0;
        for (int x = 0; x < h && f1 < 0; ++x)
            for (int y = x + 1; y < h; ++y) {
                if (cc == idx2) { f1 = x; f2 = y; break; }
                cc++;
            }
        a = hol[f1]; b = hol[f2];
    } else {
        int nha = holes_of_spin(s, d, 0, ha);
        int nhb = holes_of_spin(s, d, 1, hb);
        nh = (uint64_t)nha * (uint64_t)nhb;
        if (nh == 0) return 0;
        a = ha[idx2 / (uint64_t)nhb];
        b = hb[idx2 % (uint64_t)nhb];
    }
    det_t t = d;
    det_set(s, &t, i, 0); det_set(s, &t, j, 0); det_set(s, &t, a, 1); det_set(s, &t, b, 1);
    *tgt = t;
    double pd = 1.0 - p_single;
    *pgen = pd / (double)(npair * nh);
    return 1;
}

/* Uniform generator from one Philox block r[4]: lane 0 decides single vs
 * double, lane 1 the electron(s), lane 2 the hole(s). */
static int gen_uniform(const orc_sys *s, det_t d, const uint64_t r[4], double p_single,
                       det_t *tgt, double *pgen)
{
    int n = s->na + s->nb;
    int single = unif(r[0]) < p_single;
    if (single) {
        uint64_t idx1 = pick(r[1], (uint64_t)n);
        uint64_t c2 = orc_uniform_count2(s, d, 1, idx1);
        if (c2 == 0) return 0;
        return orc_uniform_apply(s, d, 1, idx1, pick(r[2], c2), p_single, tgt, pgen);
    }
    if (n < 2) return 0;
    uint64_t npair = (uint64_t)n * (uint64_t)(n - 1) / 2;
    uint64_t idx1 = pick(r[1], npair);
    uint64_t c2 = orc_uniform_count2(s, d, 0, idx1);
    if (c2 == 0) return 0;
    return orc_uniform_apply(s, d, 0, idx1, pick(r[2], c2), p_single, tgt, pgen);
}

/* Probability that the 32-bit choice floor(x m / 2^32), x uniform over the
 * 2^32 words, equals e: the words x >= e 2^32 / m and < (e+1) 2^32 / m,
 * counted exactly and divided by 2^32 (both exact in binary64).  It is
 * 1/m exactly when m is a power of two, and within 2^-32 of it otherwise. */
static double pick32_prob(uint64_t e, uint64_t m)
{
    uint64_t lo = ((e << 32) + m - 1) / m;
    uint64_t hi = (((e + 1) << 32) + m - 1) / m;
    return (double)(hi - lo) * 0x1.0p-32;
}

/* Real-space lattice generator.  The paper names it (Sec. II) without an
 * algorithm.  Reading: pick one of the n electrons, then one of the z_p
 * lattice neighbours of its site (the distinct q with h_pq != 0,
 * ascending), same spin; null if that orbital is occupied.  Both choices
 * are made from 32-bit words (below), so p_gen is the product of their
 * exact probabilities, p(e) p(q|e), which equals 1 / (n * z_p) whenever n
 * and z_p are powers of two.  Exact for Hubbard-type Hamiltonians, whose
 * only off-diagonal elements are hoppings along bonds. */
int orc_lattice_apply(const orc_sys *s, det_t d, uint64_t idx1, uint64_t idx2,
                      det_t *tgt, double *pgen)
{
    int occ[128];
    int n = det_occ_list(s, d, occ);
    int i = occ[idx1];
    int p = so_orb(s, i);
    int z = s->deg[p];
    if (z == 0) return 0;
    int q = s->nbr[p * s->N + (int)idx2];
    int a = so_spin(s, i) ? s->N + q : q;
    if (det_occ(s, d, a)) return 0;
    det_t t = d; det_set(s, &t, i, 0); det_set(s, &t, a, 1);
    *tgt = t;
    double pe = pick32_prob(idx1, (uint64_t)n);
    double pq = pick32_prob(idx2, (uint64_t)z);
    *pgen = pe * pq;
    return 1;
}

/* Lattice draw: electron from the high and neighbour from the low 32-bit
 * half of word 0 (Reading: one Philox block per attempt; both choices are
 * floor(x m / 2^32), whose exact probabilities enter p_gen above). */
static uint64_t pick32(uint32_t x, uint64_t m)
{
    return ((uint64_t)x * m) >> 32;
}

static int gen_lattice(const orc_sys *s, det_t d, const uint64_t r[4], det_t *tgt, double *pgen)
{
    int occ[128];
    int n = det_occ_list(s, d, occ);
    uint64_t idx1 = pick32((uint32_t)(r[0] >> 32), (uint64_t)n);
    int p = so_orb(s, occ[idx1]);
    int z = s->deg[p];
    if (z == 0) return 0;
    return orc_lattice_apply(s, d, idx1, pick32((uint32_t)r[0], (uint64_t)z), tgt, pgen);
}

int orc_lattice_degree(const orc_sys *s, int p) { return s->deg[p]; }

/* ------------------------------------------------------------------------- */
/* Walker population and the step.                                            */
/* ------------------------------------------------------------------------- */
enum { MODE_INTEGER = 0, MODE_REAL = 1 };
enum { GEN_UNIFORM = 0, GEN_LATTICE = 1, GEN_PCHB = 2, GEN_CS = 3, GEN_PE = 4 };

typedef struct {
    det_t d;
    double v;
    double diag; /* H_ii - H_00 */
} ent_t;

typedef struct {
    det_t d;
    double v;
    int init;
    int64_t par;   /* adaptive shift: the non-initiator parent's list index, else -1 */
    double habs;   /* |H_ji| of the spawn */
} rec_t;

typedef struct {
    double tau, target, n_a, c_min, zeta, p_single, p_opp;
    int interval, mode, gen;
    uint64_t seed, replica;
    double xi; /* restoring strength of the shift update; < 0: zeta^2/4 */
    int adaptive; /* adaptive shift for non-initiators (Sec. "Adaptive Shift") */
    int rechoose; /* re-choose the reference when the shift starts varying */
} orc_params;

typedef struct {
    double nw, nref, enum_, shift;
    int64_t ndets, attempts, spawns;
    int vary, bloom;
} orc_stats;

typedef struct {
    const orc_sys *s;
    orc_params p;
    det_t ref;     /* energy zero: H_00 = <ref|H|ref> */
    det_t proj;    /* reference of the projected energy (Sec. IV), always an initiator */
    int64_t t_vary; /* step at which the shift started varying (-1: not yet) */
    double h00;
    int64_t t;
    double S;
    int vary;
    int64_t t_last;
    double nw_last;
    double *nw_ring;   /* N_w(t) of the last A+1 steps, indexed t mod (A+1) */
    int64_t t_set;     /* step at which the population was last set */
    ent_t *list;
    int64_t n, cap;
    /* semi-stochastic deterministic space (Sec. "Semi-stochastic FCIQMC") */
    det_t *core;        /* nc determinants, ascending */
    int64_t nc;
    double *hcore;      /* nc x nc: H_kj for k != j (dense; the diagonal is unused) */
    double *core_diag;  /* H_kk - H_00 */
    /* discarded spawns of the last step (Sec. "Perturbative correction"):
     * targets unoccupied at tau that no initiator spawn reached, with the
     * summed weight spawned onto them; ascending */
    int collect_rej;
    det_t *rej;
    double *rej_w;
    int64_t nrej;
    double S_step;      /* shift used in the last step */
    /* adaptive shift of the last step: f of each determinant occupied at tau */
    det_t *f_det;
    double *f_val;
    int64_t nf;
    /* 2-RDM sampling (Sec. "Density matrix sampling and pure expectation
     * values"): the population the last step started from, and every
     * non-null excitation it generated with the weight C_i / (m_i p_gen) */
    int log_exc;
    ent_t *prev;
    int64_t nprev;
    det_t *exc_par, *exc_chi;
    double *exc_w;
    int64_t nexc, cexc;
} orc_run;

static int ent_cmp(const void *x, const void *y)
{
    return det_cmp(((const ent_t *)x)->d, ((const ent_t *)y)->d);
}

/* Records sort by target; ties keep emission order (parent order, then k). */
typedef struct { rec_t r; int64_t seq; } srec_t;
static int srec_cmp(const void *x, const void *y)
{
    const srec_t *a = (const srec_t *)x, *b = (const srec_t *)y;
    int c = det_cmp(a->r.d, b->r.d);
    if (c) return c;
    return a->seq < b->seq ? -1 : (a->seq > b->seq);
}

/* Random words of (determinant D, iteration t, ordinal k, purpose), from a
 * Philox4x32-10 block: counter (64-bit identity of D, t, k), key = a hash of
 * (seed, replica, purpose).  The identity of a one-word determinant is the
 * word itself; a two-word determinant (alpha, beta) is hashed to 64 bits,
 * mix(alpha xor mix(beta + c)) with the splitmix finaliser.  t and k enter
 * with their low 32 bits.  Two 64-bit words per block, word j = lanes 2j and
 * 2j+1 (low half first); draw() takes words 0-1 from the block of the purpose
 * and words 2-3 from the block of purpose + 128. */
static void draw_block(const orc_run *r, det_t d, int64_t t, uint64_t k, uint64_t purpose, uint64_t out[2])
{
    uint64_t w0, w1;
    layout_words(r->s, d, &w0, &w1);
    uint64_t id = r->s->words == 1 ? w0 : splitmix64_fin(w0 ^ splitmix64_fin(w1 + 0x632BE59BD9B4E019ULL));
    uint64_t sk = splitmix64_fin(splitmix64_fin(r->p.seed) ^ ((r->p.replica << 8) | purpose));
    uint32_t ctr[4] = {(uint32_t)id, (uint32_t)(id >> 32), (uint32_t)t, (uint32_t)k};
    uint32_t key[2] = {(uint32_t)sk, (uint32_t)(sk >> 32)}, o[4];
    orc_philox4x32_10(ctr, key, o);
    out[0] = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
    out[1] = (uint64_t)o[2] | ((uint64_t)o[3] << 32);
}

static void draw(const orc_run *r, det_t d, int64_t t, uint64_t k, int purpose, uint64_t out[4])
{
    draw_block(r, d, t, k, (uint64_t)purpose, out);
    draw_block(r, d, t, k, (uint64_t)purpose | 128, out + 2);
}

/* The random words of spawn attempt k: four words (two blocks), word 3 the
 * acceptance; the lattice generator uses one block, its electron and its
 * neighbour from the two 32-bit halves of word 0 and the acceptance from
 * word 1 (returned in word 3). */
static void spawn_words(const orc_run *r, det_t d, int64_t t, uint64_t k, uint64_t out[4])
{
    if (r->p.gen == GEN_LATTICE) {
        draw_block(r, d, t, k, PURPOSE_SPAWN, out);
        out[3] = out[1];
        out[1] = out[2] = 0;
    } else {
        draw(r, d, t, k, PURPOSE_SPAWN, out);
    }
}

orc_run *orc_run_create(const orc_sys *s, const orc_params *p, uint64_t ref_a, uint64_t ref_b)
{
    orc_run *r = (orc_run *)calloc(1, sizeof(orc_run));
    r->s = s;
    r->p = *p;
    if (r->p.xi < 0.0) {
        double z2 = r->p.zeta * r->p.zeta;
        r->p.xi = z2 / 4.0;
    }
    if (r->p.p_single < 0.0) {
        /* Appendix A.2, "Preparing for excitation generation": p_sing ~ nN/(nN + n^2 N^2) */
        double n = (double)(s->na + s->nb), N = (double)s->N;
        double nN = n * N;
        double n2N2 = nN * nN;
        r->p.p_single = nN / (nN + n2N2);
    }
    if (ref_a == 0 && ref_b == 0) {
        ref_a = (s->na == 64) ? ~0ULL : ((1ULL << s->na) - 1);
        ref_b = (s->nb == 64) ? ~0ULL : ((1ULL << s->nb) - 1);
    }
    r->ref.a = ref_a; r->ref.b = ref_b;
    r->proj = r->ref;
    r->t_vary = -1;
    r->h00 = orc_hdiag_det(s, r->ref);
    r->cap = 16;
    r->list = (ent_t *)malloc(sizeof(ent_t) * r->cap);
    r->nw_ring = (double *)calloc((size_t)r->p.interval + 1, sizeof(double));
    return r;
}

static void core_clear(orc_run *r)
{
    free(r->core); free(r->hcore); free(r->core_diag);
    r->core = NULL; r->hcore = NULL; r->core_diag = NULL;
    r->nc = 0;
}

void orc_run_free(orc_run *r)
{
    if (!r) return;
    core_clear(r);
    free(r->rej); free(r->rej_w);
    free(r->prev); free(r->exc_par); free(r->exc_chi); free(r->exc_w);
    free(r->f_det); free(r->f_val);
    free(r->list);
    free(r->nw_ring);
    free(r);
}

double orc_run_h00(const orc_run *r) { return r->h00; }
double orc_run_p_single(const orc_run *r) { return r->p.p_single; }

/* Replace the population; values are stored as given, zero entries dropped.
 * A deterministic space, if any, is dropped too. */
void orc_run_set_walkers(orc_run *r, const uint64_t *a, const uint64_t *b, const double *v, int64_t n)
{
    core_clear(r);
    free(r->list);
    r->cap = n > 16 ? n : 16;
    r->list = (ent_t *)malloc(sizeof(ent_t) * r->cap);
    r->n = 0;
    for (int64_t x = 0; x < n; ++x) {
        if (v[x] == 0.0) continue;
        ent_t e;
        e.d.a = a[x]; e.d.b = b[x]; e.v = v[x];
        e.diag = orc_hdiag_det(r->s, e.d) - r->h00;
        r->list[r->n++] = e;
    }
    qsort(r->list, r->n, sizeof(ent_t), ent_cmp);
    double nw = 0.0;
    for (int64_t x = 0; x < r->n; ++x) nw = nw + fabs(r->list[x].v);
    r->t_set = r->t;
    r->nw_ring[r->t % (r->p.interval + 1)] = nw;
}

void orc_run_set_state(orc_run *r, int64_t t, double S, int vary, int64_t t_last, double nw_last)
{
    /* re-key the growth history to the new step counter */
    double nw0 = r->nw_ring[r->t % (r->p.interval + 1)];
    r->t = t; r->S = S; r->vary = vary; r->t_last = t_last; r->nw_last = nw_last;
    r->t_set = t;
    r->nw_ring[t % (r->p.interval + 1)] = nw0;
}

void orc_run_get_state(const orc_run *r, int64_t *t, double *S, int *vary, int64_t *t_last,
                       double *nw_last)
{
    *t = r->t; *S = r->S; *vary = r->vary; *t_last = r->t_last; *nw_last = r->nw_last;
}

int64_t orc_run_size(const orc_run *r) { return r->n; }

void orc_run_get_walkers(const orc_run *r, uint64_t *a, uint64_t *b, double *v, double *diag)
{
    for (int64_t x = 0; x < r->n; ++x) {
        a[x] = r->list[x].d.a; b[x] = r->list[x].d.b; v[x] = r->list[x].v;
        if (diag) diag[x] = r->list[x].diag;
    }
}

static int64_t find(const ent_t *list, int64_t n, det_t d)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        int c = det_cmp(list[mid].d, d);
        if (c == 0) return mid;
        if (c < 0) lo = mid + 1; else hi = mid;
    }
    return -1;
}

/* Index of d in the deterministic space, -1 if it is not there. */
static int64_t core_find(const orc_run *r, det_t d)
{
    int64_t lo = 0, hi = r->nc;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        int c = det_cmp(r->core[mid], d);
        if (c == 0) return mid;
        if (c < 0) lo = mid + 1; else hi = mid;
    }
    return -1;
}

/* Order for choosing the deterministic space: larger |C| first, ties by
 * ascending determinant. */
static int weight_cmp(const void *x, const void *y)
{
    const ent_t *p = (const ent_t *)x, *q = (const ent_t *)y;
    double a = fabs(p->v), b = fabs(q->v);
    if (a != b) return a > b ? -1 : 1;
    return det_cmp(p->d, q->d);
}

static int detv_cmp(const void *x, const void *y) { return det_cmp(*(const det_t *)x, *(const det_t *)y); }

/* Semi-stochastic projection (Sec. "Semi-stochastic FCIQMC"): the projector
 * splits into P^D, its elements between determinants of the deterministic
 * space D, applied exactly every step as a matrix-vector product, and the
 * rest, sampled by spawning as usual.  D is the n_core most populated
 * determinants of the current population (the paper's usual choice); it is
 * ordered by determinant and H^D is stored with it.  Readings (the paper
 * leaves them open): P^D includes the diagonal, so the determinants of D
 * have no stochastic death; their coefficients are never compressed to
 * C_min and they stay in the population at any value, zero included; they
 * count as initiators; spawns from D into D are dropped (their terms are in
 * P^D).  Real coefficients only.  Returns the size of D, -1 in integer mode. */
int64_t orc_run_set_core(orc_run *r, int64_t n_core)
{
    core_clear(r);
    if (r->p.mode != MODE_REAL) return -1;
    int64_t nc = n_core < r->n ? n_core : r->n;
    if (nc <= 0) return 0;
    ent_t *tmp = (ent_t *)malloc(sizeof(ent_t) * r->n);
    memcpy(tmp, r->list, sizeof(ent_t) * r->n);
    qsort(tmp, r->n, sizeof(ent_t), weight_cmp);
    r->core = (det_t *)malloc(sizeof(det_t) * nc);
    for (int64_t k = 0; k < nc; ++k) r->core[k] = tmp[k].d;
    free(tmp);
    qsort(r->core, nc, sizeof(det_t), detv_cmp);
    r->nc = nc;
    r->hcore = (double *)calloc((size_t)(nc * nc), sizeof(double));
    r->core_diag = (double *)malloc(sizeof(double) * nc);
    for (int64_t k = 0; k < nc; ++k) {
        r->core_diag[k] = r->list[find(r->list, r->n, r->core[k])].diag;
        for (int64_t j = 0; j < nc; ++j)
            if (j != k) r->hcore[k * nc + j] = orc_hij_det(r->s, r->core[j], r->core[k]);
    }
    return nc;
}

int64_t orc_run_core_size(const orc_run *r) { return r->nc; }

void orc_run_get_core(const orc_run *r, uint64_t *a, uint64_t *b)
{
    for (int64_t k = 0; k < r->nc; ++k) { a[k] = r->core[k].a; b[k] = r->core[k].b; }
}

void orc_run_collect_rejected(orc_run *r, int on) { r->collect_rej = on; }

/* Epstein-Nesbet second-order correction from the spawns discarded on both
 * replicas in their last step (Sec. "Perturbative correction", Eq.
 * (pt2_correction)), before the normalisation by the replica overlap
 * (orc_pair_overlap):
 *   dE2 = 1/dtau^2 sum_j S_j^1 S_j^2 / (E_0 - H_jj)
 * over the determinants j rejected by both, S_j^r the weight spawned onto j
 * in replica r.  Reading: E_0 is the mean of the two replicas' shifts in
 * that step; energies relative to H_00 (E_0 - H_jj = S - (H_jj - H_00)). */
double orc_pair_pt2(const orc_run *r1, const orc_run *r2)
{
    double e0 = (r1->S_step + r2->S_step) / 2.0;
    double tau2 = r1->p.tau * r1->p.tau;
    double acc = 0.0;
    int64_t x = 0, y = 0;
    while (x < r1->nrej && y < r2->nrej) {
        int c = det_cmp(r1->rej[x], r2->rej[y]);
        if (c < 0) { ++x; continue; }
        if (c > 0) { ++y; continue; }
        double dj = orc_hdiag_det(r1->s, r1->rej[x]) - r1->h00;
        double num = r1->rej_w[x] * r2->rej_w[y];
        double den = e0 - dj;
        double q = num / den;
        acc = acc + q;
        ++x; ++y;
    }
    return acc / tau2;
}

/* Overlap of two replicas' populations, sum_i C_i^1 C_i^2: the norm of the
 * replica estimate of the wave function.  Reading: Eq. (pt2_correction)
 * holds for a normalised wave function, so dE2 is divided by this overlap of
 * the populations the step started from (averaged as a ratio of means over
 * steps), as the variational energy it corrects is. */
double orc_pair_overlap(const orc_run *r1, const orc_run *r2)
{
    double acc = 0.0;
    int64_t x = 0, y = 0;
    while (x < r1->n && y < r2->n) {
        int c = det_cmp(r1->list[x].d, r2->list[y].d);
        if (c < 0) { ++x; continue; }
        if (c > 0) { ++y; continue; }
        double q = r1->list[x].v * r2->list[y].v;
        acc = acc + q;
        ++x; ++y;
    }
    return acc;
}

/* ------------------------------------------------------------------------- */
/* Two-body reduced density matrix (Sec. "Density matrix sampling and pure   */
/* expectation values", Eq. (FCI2RDM)):                                        */
/*   Gamma_{kl,mn} = sum_{i,j} C_i^A C_j^B <D_i| a+_k a+_l a_n a_m |D_j>      */
/* over spin orbitals in canonical order.  It is antisymmetric in (k,l) and  */
/* in (m,n), so only k < l, m < n are kept: pair index                        */
/* P(k,l) = k(2K-k-1)/2 + l-k-1 over the M = K(K-1)/2 pairs of the K = 2N     */
/* spin orbitals, stored row-major as G[P(k,l) M + P(m,n)].                   */
/* ------------------------------------------------------------------------- */
int64_t orc_rdm_dim(const orc_sys *s)
{
    int64_t K = 2 * (int64_t)s->N;
    return K * (K - 1) / 2;
}

static int64_t rdm_pair(int64_t K, int k, int l)
{
    return (int64_t)k * (2 * K - k - 1) / 2 + (l - k - 1);
}

/* <D_i| a+_k a+_l a_n a_m |D_j>: the operators applied to D_j right to left
 * (a_m first); 0 unless the result is D_i, else the fermion sign. */
static int rdm_element(const orc_sys *s, det_t di, det_t dj, int k, int l, int m, int n)
{
    det_t t = dj;
    if (!det_occ(s, t, m)) return 0;
    int par = op_annihilate(s, &t, m);
    if (!det_occ(s, t, n)) return 0;
    par ^= op_annihilate(s, &t, n);
    if (det_occ(s, t, l)) return 0;
    par ^= op_create(s, &t, l);
    if (det_occ(s, t, k)) return 0;
    par ^= op_create(s, &t, k);
    if (!det_eq(t, di)) return 0;
    return par ? -1 : 1;
}

/* G += coef <D_i| a+_k a+_l a_n a_m |D_j> for every k<l, m<n (ascending m,
 * n, then k, l), each addition one rounding. */
static void rdm_add(const orc_sys *s, det_t di, det_t dj, double coef, double *G)
{
    int K = 2 * s->N;
    int64_t M = (int64_t)K * (K - 1) / 2;
    for (int m = 0; m < K; ++m)
        for (int n = m + 1; n < K; ++n) {
            if (!det_occ(s, dj, m) || !det_occ(s, dj, n)) continue;
            for (int k = 0; k < K; ++k)
                for (int l = k + 1; l < K; ++l) {
                    /* the created orbitals are occupied in the result */
                    if (!det_occ(s, di, k) || !det_occ(s, di, l)) continue;
                    int sg = rdm_element(s, di, dj, k, l, m, n);
                    if (sg == 0) continue;
                    double x = sg > 0 ? coef : -coef;
                    int64_t at = rdm_pair(K, k, l) * M + rdm_pair(K, m, n);
                    G[at] = G[at] + x;
                }
        }
}

/* The definition over a state pair on one determinant list: D_i, D_j run
 * over the list (a, b masks; ascending), C^A = ca, C^B = cb.  G (M x M) is
 * added to. */
void orc_rdm_exact(const orc_sys *s, const uint64_t *a, const uint64_t *b, const double *ca,
                   const double *cb, int64_t n, double *G)
{
    for (int64_t j = 0; j < n; ++j) {
        if (cb[j] == 0.0) continue;
        det_t dj = {a[j], b[j]};
        for (int64_t i = 0; i < n; ++i) {
            if (ca[i] == 0.0) continue;
            det_t di = {a[i], b[i]};
            int x = __builtin_popcountll(di.a ^ dj.a) + __builtin_popcountll(di.b ^ dj.b);
            if (x > 4) continue;  /* no two-body operator connects them */
            double c = ca[i] * cb[j];
            rdm_add(s, di, dj, c, G);
        }
    }
}

/* Energy of a 2-RDM, <A|H|B>/<A|B> + E_core, from the textbook contraction
 *   E = sum_pq h_pq gamma_pq + sum_{k<l, m<n} Gamma_{kl,mn} <kl||mn>,
 * <kl||mn> = <kl|mn> - <kl|nm>, <kl|mn> = (km|ln) d(s_k,s_m) d(s_l,s_n), and
 * the one-body matrix gamma_pq = sum_r Gamma_{pr,qr} / (n-1) (n electrons).
 * The norm <A|B> is the trace sum_{k<l} Gamma_{kl,kl} / (n(n-1)/2), returned
 * in *norm.  Sums in ascending index order. */
double orc_rdm_energy(const orc_sys *s, const double *G, double *norm)
{
    int K = 2 * s->N, N = s->N;
    int ne = s->na + s->nb;
    int64_t M = (int64_t)K * (K - 1) / 2;
    double tr = 0.0;
    for (int64_t P = 0; P < M; ++P) tr = tr + G[P * M + P];
    double npair = (double)ne * (double)(ne - 1) / 2.0;
    *norm = tr / npair;
    /* one-body part */
    double e1 = 0.0;
    for (int p = 0; p < K; ++p)
        for (int q = 0; q < K; ++q) {
            if (so_spin(s, p) != so_spin(s, q)) continue;
            double g = 0.0;
            for (int r = 0; r < K; ++r) {
                if (r == p || r == q) continue;
                /* Gamma_{pr,qr} from the stored k<l, m<n entry */
                int sg = 1;
                int k = p, l = r, m = q, n = r;
                if (k > l) { int t = k; k = l; l = t; sg = -sg; }
                if (m > n) { int t = m; m = n; n = t; sg = -sg; }
                double v = G[rdm_pair(K, k, l) * M + rdm_pair(K, m, n)];
                g = g + (sg > 0 ? v : -v);
            }
            double gam = g / (double)(ne - 1);
            double x = s->h[so_orb(s, p) * N + so_orb(s, q)] * gam;
            e1 = e1 + x;
        }
    /* two-body part */
    double e2 = 0.0;
    for (int k = 0; k < K; ++k)
        for (int l = k + 1; l < K; ++l)
            for (int m = 0; m < K; ++m)
                for (int n = m + 1; n < K; ++n) {
                    double v = G[rdm_pair(K, k, l) * M + rdm_pair(K, m, n)];
                    if (v == 0.0) continue;
                    double d = (so_spin(s, k) == so_spin(s, m) && so_spin(s, l) == so_spin(s, n))
                                   ? eri(s, so_orb(s, k), so_orb(s, m), so_orb(s, l), so_orb(s, n)) : 0.0;
                    double x = (so_spin(s, k) == so_spin(s, n) && so_spin(s, l) == so_spin(s, m))
                                   ? eri(s, so_orb(s, k), so_orb(s, n), so_orb(s, l), so_orb(s, m)) : 0.0;
                    double a = d - x;
                    double c = v * a;
                    e2 = e2 + c;
                }
    double e = e1 + e2;
    double q = e / *norm;
    return q + s->e_core;
}

void orc_run_log_excitations(orc_run *r, int on) { r->log_exc = on; }

void orc_run_get_proj(const orc_run *r, uint64_t *a, uint64_t *b)
{
    *a = r->proj.a;
    *b = r->proj.b;
}
int64_t orc_run_excitations(const orc_run *r) { return r->nexc; }

static double prev_value(const orc_run *r, det_t d)
{
    int64_t at = find(r->prev, r->nprev, d);
    return at >= 0 ? r->prev[at].v : 0.0;
}

/* One paired step's sample of the replica 2-RDM (Sec. "Density matrix
 * sampling and pure expectation values": the replica trick makes the
 * estimate bilinear in two independent populations), added to G:
 *  - the diagonal terms i = j exactly: C_i^1 C_i^2 over the determinants
 *    occupied in both populations the step started from;
 *  - the off-diagonal terms from the excitations the step generated: an
 *    excitation D_i -> D_j drawn by replica r from the population at tau
 *    (m_i attempts on D_i, each producing D_j with probability p_gen) adds
 *    C_i^r C_j^r' / (m_i p_gen) times the operator elements
 *    <D_i|a+_k a+_l a_n a_m|D_j> (r' the other replica; C_j^r' its
 *    coefficient at tau), whose expectation is the sum over all j of
 *    C_i^r C_j^r' <D_i|...|D_j>.  Each replica's parents estimate one
 *    ordering of the replica product; both are added with weight 1/2.
 *    Readings: every non-null draw counts, accepted or not, and the
 *    unnormalised, not yet hermitian sum is returned (the paper makes the
 *    accumulated matrix hermitian and fixes its trace at the end).
 * Order: diagonal by ascending determinant, then replica 1's excitations in
 * generation order, then replica 2's. */
void orc_pair_rdm_step(const orc_run *r1, const orc_run *r2, double *G)
{
    const orc_sys *s = r1->s;
    int64_t x = 0, y = 0;
    while (x < r1->nprev && y < r2->nprev) {
        int c = det_cmp(r1->prev[x].d, r2->prev[y].d);
        if (c < 0) { ++x; continue; }
        if (c > 0) { ++y; continue; }
        double q = r1->prev[x].v * r2->prev[y].v;
        if (q != 0.0) rdm_add(s, r1->prev[x].d, r1->prev[x].d, q, G);
        ++x; ++y;
    }
    const orc_run *rr[2] = {r1, r2};
    for (int side = 0; side < 2; ++side) {
        const orc_run *r = rr[side], *o = rr[1 - side];
        for (int64_t e = 0; e < r->nexc; ++e) {
            double cj = prev_value(o, r->exc_chi[e]);
            if (cj == 0.0) continue;
            double w1 = r->exc_w[e] * cj;
            double w2 = w1 * 0.5;
            rdm_add(s, r->exc_par[e], r->exc_chi[e], w2, G);
        }
    }
}

int64_t orc_run_rejected_size(const orc_run *r) { return r->nrej; }

/* f of determinant (a, b) in the last adaptive-shift step (1 for an
 * initiator or a determinant without spawn weight); -1 if it was not
 * occupied at the start of that step. */
double orc_run_adaptive_f(const orc_run *r, uint64_t a, uint64_t b)
{
    for (int64_t x = 0; x < r->nf; ++x)
        if (r->f_det[x].a == a && r->f_det[x].b == b) return r->f_val[x];
    return -1.0;
}

void orc_run_get_rejected(const orc_run *r, uint64_t *a, uint64_t *b, double *w)
{
    for (int64_t x = 0; x < r->nrej; ++x) { a[x] = r->rej[x].a; b[x] = r->rej[x].b; w[x] = r->rej_w[x]; }
}

/* Stochastic compression to C_min (Sec. I, the compressed storage rule):
 * keep |x| >= C_min, else sign(x) C_min with probability |x|/C_min, else 0. */
static double round_cmin(double x, double cmin, double u)
{
    double ax = fabs(x);
    if (ax >= cmin || x == 0.0) return x;
    double pr = ax / cmin;
    if (u < pr) return x < 0.0 ? -cmin : cmin;
    return 0.0;
}

int orc_pchb_gen(const orc_sys *s, det_t d, const uint64_t r1[4],
                 double p_single, double p_opp, det_t *tgt, double *pgen);
int orc_cs_gen(const orc_sys *s, det_t d, const uint64_t r1[4], const uint64_t r2[4],
               double p_single, double p_opp, int exact, det_t *tgt, double *pgen);

/* One imaginary-time step, Eq. (projector) split as Eq. (fciqmc_dyn):
 * (a) spawning from C(tau), (b) death in place, (c) annihilation with the
 * initiator rule; then the estimators and the shift update. */
int orc_run_step(orc_run *r, orc_stats *st)
{
    const orc_sys *s = r->s;
    const orc_params *p = &r->p;
    int64_t t = r->t;
    int integer = p->mode == MODE_INTEGER;
    memset(st, 0, sizeof(*st));

    if (r->log_exc) {
        free(r->prev);
        r->prev = (ent_t *)malloc(sizeof(ent_t) * (r->n > 0 ? r->n : 1));
        memcpy(r->prev, r->list, sizeof(ent_t) * (size_t)r->n);
        r->nprev = r->n;
        r->nexc = 0;
    }

    /* (a) spawning.  Every walker of every occupied determinant makes one
     * attempt (integer mode: |C_i| attempts; real mode: ceil(|C_i|)).
     * Attempt k of determinant D_i draws Philox block (D_i, t, k, SPAWN). */
    int64_t rcap = 1024, nrec = 0;
    srec_t *recs = (srec_t *)malloc(sizeof(srec_t) * rcap);
    for (int64_t x = 0; x < r->n; ++x) {
        const ent_t *e = &r->list[x];
        double C = e->v;
        double aC = fabs(C);
        int64_t m = integer ? (int64_t)aC : (int64_t)ceil(aC);
        /* initiator: |C_i| above n_a (Sec. I); Reading: the reference always
         * counts as one; a negative n_a switches the approximation off. */
        int init = (p->n_a < 0.0) || (aC > p->n_a) || det_eq(e->d, r->proj);
        int pcore = r->nc > 0 && core_find(r, e->d) >= 0;
        if (pcore) init = 1;
        st->attempts += m;
        for (int64_t k = 0; k < m; ++k) {
            uint64_t rr[4];
            spawn_words(r, e->d, t, (uint64_t)k, rr);
            det_t tgt;
            double pgen;
            int ok;
            if (p->gen == GEN_UNIFORM) ok = gen_uniform(s, e->d, rr, p->p_single, &tgt, &pgen);
            else if (p->gen == GEN_LATTICE) ok = gen_lattice(s, e->d, rr, &tgt, &pgen);
            else if (p->gen == GEN_PCHB) ok = orc_pchb_gen(s, e->d, rr, p->p_single, p->p_opp, &tgt, &pgen);
            else {
                uint64_t r2[4] = {0, 0, 0, 0};
                draw_block(r, e->d, t, (uint64_t)k, PURPOSE_SPAWN2, r2);  /* words 0-1 */
                ok = orc_cs_gen(s, e->d, rr, r2, p->p_single, p->p_opp, p->gen == GEN_PE, &tgt, &pgen);
            }
            if (!ok) continue;
            if (r->log_exc) {
                /* every generated excitation, accepted or not, with the
                 * inverse of its expected number of draws in this step */
                if (r->nexc == r->cexc) {
                    r->cexc = r->cexc ? 2 * r->cexc : 1024;
                    r->exc_par = (det_t *)realloc(r->exc_par, sizeof(det_t) * r->cexc);
                    r->exc_chi = (det_t *)realloc(r->exc_chi, sizeof(det_t) * r->cexc);
                    r->exc_w = (double *)realloc(r->exc_w, sizeof(double) * r->cexc);
                }
                double d1 = pgen * (double)m;
                r->exc_par[r->nexc] = e->d;
                r->exc_chi[r->nexc] = tgt;
                r->exc_w[r->nexc] = C / d1;
                r->nexc++;
            }
            if (pcore && core_find(r, tgt) >= 0) continue;  /* in P^D */
            double H = orc_hij_det(s, e->d, tgt);
            if (H == 0.0) continue;
            double amt;
            if (integer) {
                /* p_s = dtau |H_ij| / p_gen (Sec. II); the integer part spawns
                 * deterministically, the fraction with that probability. */
                double num = p->tau * fabs(H);
                double ps = num / pgen;
                double fl = floor(ps);
                double fr = ps - fl;
                double nn = fl + (unif(rr[3]) < fr ? 1.0 : 0.0);
                if (nn == 0.0) continue;
                if (nn > 1073741824.0) st->bloom = 1;
                /* Reading: the child's sign is -sgn(H_ji) sgn(C_i), the sign of
                 * the off-diagonal term -dtau H_ji C_i of Eq. (projector); the
                 * "+" printed under the spawn term of Eq. (fciqmc_dyn) is taken
                 * as a typo. */
                amt = ((H > 0.0) == (C > 0.0)) ? -nn : nn;
            } else {
                double x1 = p->tau * H;
                double x2 = x1 * C;
                double d1 = pgen * (double)m;
                double amp = -(x2 / d1);
                amt = round_cmin(amp, p->c_min, unif(rr[3]));
                if (amt == 0.0) continue;
            }
            if (nrec == rcap) {
                rcap *= 2;
                recs = (srec_t *)realloc(recs, sizeof(srec_t) * rcap);
            }
            recs[nrec].r.d = tgt;
            recs[nrec].r.v = amt;
            recs[nrec].r.init = init;
            recs[nrec].r.par = (p->adaptive && !init) ? x : -1;
            recs[nrec].r.habs = fabs(H);
            recs[nrec].seq = nrec;
            nrec++;
        }
    }
    st->spawns = nrec;

    /* Adaptive shift (Sec. "Adaptive Shift", Eq. (as_fval)): a non-initiator
     * D_i dies with the local shift S_i = f_i S, f_i the share of the weights
     * w_ij = |H_ij| / (H_jj - E_0) of its spawns this step that the
     * initiator rule accepted (target occupied at tau).  Readings: E_0 is the
     * current shift, the denominator is taken as |H_jj - E_0| (weight 0 if
     * it vanishes) and w is capped at 1e6; every spawn record counts once;
     * f_i = 1 when no weight was spawned; the weights are summed in fixed
     * point with 2^-40 resolution, so the sums do not depend on their order. */
    int64_t *acc_w = NULL, *all_w = NULL;
    if (p->adaptive) {
        free(r->f_det); free(r->f_val);
        r->f_det = (det_t *)malloc(sizeof(det_t) * (r->n > 0 ? r->n : 1));
        r->f_val = (double *)malloc(sizeof(double) * (r->n > 0 ? r->n : 1));
        r->nf = r->n;
        acc_w = (int64_t *)calloc((size_t)(r->n > 0 ? r->n : 1), sizeof(int64_t));
        all_w = (int64_t *)calloc((size_t)(r->n > 0 ? r->n : 1), sizeof(int64_t));
        for (int64_t q = 0; q < nrec; ++q) {
            const rec_t *x = &recs[q].r;
            if (x->par < 0) continue;
            int64_t at = find(r->list, r->n, x->d);
            double dj = at >= 0 ? r->list[at].diag : orc_hdiag_det(s, x->d) - r->h00;
            double den = fabs(dj - r->S);
            double w = den > 0.0 ? x->habs / den : 0.0;
            if (w > 1e6) w = 1e6;
            int64_t qw = (int64_t)floor(w * 1099511627776.0 + 0.5);
            all_w[x->par] += qw;
            if (at >= 0) acc_w[x->par] += qw;
        }
    }

    /* (b) death: C_i <- (1 - dtau (H_ii - S)) C_i, then stochastic rounding
     * (integer mode: to the neighbouring integers; real mode: the C_min rule). */
    double *post = (double *)malloc(sizeof(double) * (r->n > 0 ? r->n : 1));
    for (int64_t x = 0; x < r->n; ++x) {
        const ent_t *e = &r->list[x];
        if (r->nc > 0 && core_find(r, e->d) >= 0) continue;  /* set below */
        double Sx = r->S;
        if (p->adaptive) {
            double ax = fabs(e->v);
            int ini = (p->n_a < 0.0) || (ax > p->n_a) || det_eq(e->d, r->proj);
            double f = 1.0;
            if (!ini && all_w[x] > 0) {
                f = (double)acc_w[x] / (double)all_w[x];
                Sx = f * r->S;
            }
            r->f_det[x] = e->d;
            r->f_val[x] = f;
        }
        double t1 = e->diag - Sx;
        double t2 = p->tau * t1;
        double f = 1.0 - t2;
        double xv = f * e->v;
        uint64_t rr[4];
        draw_block(r, e->d, t, 0, PURPOSE_DEATH, rr);
        double u = unif(rr[0]);
        if (integer) {
            double ax = fabs(xv);
            double fl = floor(ax);
            double fr = ax - fl;
            double nn = fl + (u < fr ? 1.0 : 0.0);
            post[x] = xv < 0.0 ? -nn : nn;
        } else {
            post[x] = round_cmin(xv, p->c_min, u);
        }
    }

    /* Deterministic space: (P^D C)_k = (1 - dtau (H_kk - S)) C_k
     * - dtau sum_{j != k} H_kj C_j, exactly, over j in ascending order. */
    if (r->nc > 0) {
        int64_t *at = (int64_t *)malloc(sizeof(int64_t) * r->nc);
        for (int64_t k = 0; k < r->nc; ++k) at[k] = find(r->list, r->n, r->core[k]);
        for (int64_t k = 0; k < r->nc; ++k) {
            double t1 = r->core_diag[k] - r->S;
            double t2 = p->tau * t1;
            double f = 1.0 - t2;
            double acc = f * r->list[at[k]].v;
            for (int64_t j = 0; j < r->nc; ++j) {
                if (j == k) continue;
                double x1 = p->tau * r->hcore[k * r->nc + j];
                double x2 = x1 * r->list[at[j]].v;
                acc = acc - x2;
            }
            post[at[k]] = acc;
        }
        free(at);
    }

    if (r->collect_rej) {
        free(r->rej); free(r->rej_w);
        r->rej = (det_t *)malloc(sizeof(det_t) * (nrec > 0 ? nrec : 1));
        r->rej_w = (double *)malloc(sizeof(double) * (nrec > 0 ? nrec : 1));
        r->nrej = 0;
    }
    r->S_step = r->S;

    /* (c) annihilation.  Sum all contributions per target.  Initiator rule
     * (Sec. I): matrix elements between non-initiators and determinants with
     * C(tau) = 0 are zeroed, i.e. a target unoccupied at tau only receives the
     * contributions of initiator parents; an occupied target receives all. */
    qsort(recs, nrec, sizeof(srec_t), srec_cmp);
    int64_t ncap = r->n + nrec + 1;
    ent_t *next = (ent_t *)malloc(sizeof(ent_t) * ncap);
    int64_t nn = 0;
    for (int64_t x = 0; x < r->n; ++x) {
        next[nn] = r->list[x];
        next[nn].v = post[x];
        nn++;
    }
    int64_t n_old = nn;
    for (int64_t x = 0; x < nrec;) {
        int64_t y = x;
        double sum_all = 0.0, sum_init = 0.0;
        int any_init = 0;
        while (y < nrec && det_eq(recs[y].r.d, recs[x].r.d)) {
            sum_all = sum_all + recs[y].r.v;
            if (recs[y].r.init) { sum_init = sum_init + recs[y].r.v; any_init = 1; }
            y++;
        }
        int64_t at = find(r->list, r->n, recs[x].r.d);
        if (r->collect_rej && at < 0 && !any_init) {
            r->rej[r->nrej] = recs[x].r.d;
            r->rej_w[r->nrej] = sum_all;
            r->nrej++;
        }
        if (at >= 0) {
            next[at].v = next[at].v + sum_all;
        } else if (sum_init != 0.0) {
            next[nn].d = recs[x].r.d;
            next[nn].v = sum_init;
            next[nn].diag = orc_hdiag_det(s, recs[x].r.d) - r->h00;
            nn++;
        }
        x = y;
    }
    (void)n_old;
    if (!integer) {
        for (int64_t x = 0; x < nn; ++x) {
            double v = next[x].v;
            if (v != 0.0 && fabs(v) < p->c_min && !(r->nc > 0 && core_find(r, next[x].d) >= 0)) {
                uint64_t rr[4];
                draw_block(r, next[x].d, t, 0, PURPOSE_ANN, rr);
                next[x].v = round_cmin(v, p->c_min, unif(rr[0]));
            }
        }
    }
    int64_t m = 0;
    for (int64_t x = 0; x < nn; ++x)
        if (next[x].v != 0.0 || (r->nc > 0 && core_find(r, next[x].d) >= 0)) next[m++] = next[x];
    qsort(next, m, sizeof(ent_t), ent_cmp);
    free(r->list);
    free(post);
    free(recs);
    free(acc_w);
    free(all_w);
    r->list = next;
    r->n = m;
    r->cap = ncap;
    r->t = t + 1;

    /* Estimators: walker number N_w = sum |C_i|; projected energy
     * E_Ref = <D_ref|H|Psi>/<D_ref|Psi> (Sec. IV, Eq. (proje)), kept as
     * numerator sum_{j != ref} H_ref,j C_j and denominator C_ref. */
    double nw = 0.0, nref = 0.0, en = 0.0;
    for (int64_t x = 0; x < r->n; ++x) {
        const ent_t *e = &r->list[x];
        nw = nw + fabs(e->v);
        if (det_eq(e->d, r->proj)) { nref = e->v; continue; }
        int lvl = __builtin_popcountll(e->d.a ^ r->proj.a) + __builtin_popcountll(e->d.b ^ r->proj.b);
        if (lvl == 2 || lvl == 4) {
            double h = orc_hij_det(s, r->proj, e->d);
            double c = h * e->v;
            en = en + c;
        }
    }

    /* Shift update.  The paper only says S is updated to match the ground-state
     * energy (Sec. I).  Reading: S is 0 (relative to H_00) until N_w first
     * reaches the target N_t.  At that step T, S is set from the measured
     * growth rate, S = -ln(N_w(T)/N_w(T-L))/(L dtau), with L = min(A, steps
     * since the population was set).  From then on, every A steps,
     *   S <- S - zeta/(A dtau) ln(N_w(t)/N_w(t-A)) - xi/(A dtau) ln(N_w(t)/N_t),
     * the damped population control of the original FCIQMC method with the
     * restoring term of Yang, Pahl and Brand (J. Chem. Phys. 153, 174103
     * (2020)), xi = zeta^2/4 by default.  An extinct population (N_w = 0)
     * leaves S unchanged. */
    int64_t T = r->t;
    int64_t A = (int64_t)p->interval;
    if (!r->vary) {
        if (nw >= p->target) {
            r->vary = 1;
            int64_t L = T - r->t_set;
            if (L > A) L = A;
            if (L > 0) {
                double nw_prev = r->nw_ring[(T - L) % (A + 1)];
                double c = 1.0 / ((double)L * p->tau);
                double ratio = nw / nw_prev;
                double l = log(ratio);
                double dS = c * l;
                r->S = 0.0 - dS;
            }
            r->t_last = T;
            r->nw_last = nw;
            r->t_vary = T;
        }
    } else if (T - r->t_last == A && nw > 0.0) {
        double at = (double)p->interval * p->tau;
        double c1 = p->zeta / at;
        double c2 = r->p.xi / at;
        double l1 = log(nw / r->nw_last);
        double l2 = log(nw / p->target);
        double d1 = c1 * l1;
        double d2 = c2 * l2;
        double s1 = r->S - d1;
        r->S = s1 - d2;
        r->t_last = T;
        r->nw_last = nw;
    }
    r->nw_ring[T % (A + 1)] = nw;

    /* Reference of the projected energy (Sec. IV: an appropriate reference
     * determinant).  Reading: with re-choice on, once the population has
     * relaxed for ceil(1/dtau) steps after the shift started varying, the
     * most populated determinant becomes the reference for the following
     * steps (largest |C|; ties: ascending alpha, then beta string); H_00
     * stays the energy zero of the diagonal and the shift. */
    if (p->rechoose && r->t_vary >= 0 && T == r->t_vary + (int64_t)ceil(1.0 / p->tau) && r->n > 0) {
        int64_t best = 0;
        for (int64_t x = 1; x < r->n; ++x) {
            double ax = fabs(r->list[x].v), ab = fabs(r->list[best].v);
            if (ax > ab) best = x;  /* the list is ascending: the first of equals wins */
        }
        r->proj = r->list[best].d;
    }

    st->nw = nw; st->nref = nref; st->enum_ = en; st->shift = r->S;
    st->ndets = r->n; st->vary = r->vary;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Pre-computed heat-bath (PCHB) doubles (Appendix A.3, pre-computed heat-bath  */
/* sampling), Eq. (hbs): p(ab|ij) = |H_ij^ab| / sum_a'b' |H_ij^a'b'|, drawn by */
/* Walker's alias method in O(1).                                             */
/* Reading, over spatial orbitals (no p_exch split):                          */
/*   opposite spin, electrons (I alpha, J beta) -> holes (A alpha, B beta):   */
/*       row (I,J), column A*N+B, weight |(AI|BJ)|, zero if A=I or B=J;       */
/*   same spin, electrons I<J -> holes A<B of the same spin:                  */
/*       row and column lexicographic pairs, weight |(AI|BJ) - (AJ|BI)|,      */
/*       zero if {A,B} meets {I,J}.                                           */
/* Electron pairs are uniform within their class; the class is opposite spin */
/* with probability p_opp.  A draw is null if a hole is occupied or if the    */
/* row sums to zero.  Singles are uniform, as in the uniform generator.       */
/* Random words (two blocks): [0] single/double and, beyond p_single, the    */
/* pair class; [1] electron pair; [2] alias column and, from the fraction    */
/* its pick leaves, the alias coin; [3] acceptance.                           */
/* ------------------------------------------------------------------------- */

/* Alias table by Vose's construction with LIFO work lists filled in
 * ascending column order:  scaled_c = (w_c K) / sum; while both lists are
 * non-empty pop s (small) and l (large): prob_s = scaled_s, alias_s = l,
 * scaled_l = (scaled_l + scaled_s) - 1, and l goes back to the small list if
 * scaled_l < 1, else to the large list.  Left-overs get prob 1. */
static void alias_build(const double *w, int K, double sum, double *prob, int *alias,
                        int *small, int *large, double *scaled)
{
    int ns = 0, nl = 0;
    if (sum == 0.0) {
        for (int c = 0; c < K; ++c) { prob[c] = 0.0; alias[c] = c; }
        return;
    }
    for (int c = 0; c < K; ++c) {
        double x = w[c] * (double)K;
        scaled[c] = x / sum;
        alias[c] = c;
        if (scaled[c] < 1.0) small[ns++] = c; else large[nl++] = c;
    }
    while (ns > 0 && nl > 0) {
        int s_ = small[--ns];
        int l = large[--nl];
        prob[s_] = scaled[s_];
        alias[s_] = l;
        double t = scaled[l] + scaled[s_];
        scaled[l] = t - 1.0;
        if (scaled[l] < 1.0) small[ns++] = l; else large[nl++] = l;
    }
    while (nl > 0) { int l = large[--nl]; prob[l] = 1.0; alias[l] = l; }
    while (ns > 0) { int s_ = small[--ns]; prob[s_] = 1.0; alias[s_] = s_; }
}

void orc_pchb_build(orc_sys *s)
{
    int N = s->N;
    int np = N * (N - 1) / 2;
    int NN = N * N;
    free(s->hb_w_same); free(s->hb_w_opp); free(s->hb_sum_same); free(s->hb_sum_opp);
    free(s->hb_p_same); free(s->hb_p_opp); free(s->hb_a_same); free(s->hb_a_opp);
    s->hb_w_same = (double *)calloc((size_t)np * np + 1, sizeof(double));
    s->hb_p_same = (double *)calloc((size_t)np * np + 1, sizeof(double));
    s->hb_a_same = (int *)calloc((size_t)np * np + 1, sizeof(int));
    s->hb_sum_same = (double *)calloc(np + 1, sizeof(double));
    s->hb_w_opp = (double *)calloc((size_t)NN * NN, sizeof(double));
    s->hb_p_opp = (double *)calloc((size_t)NN * NN, sizeof(double));
    s->hb_a_opp = (int *)calloc((size_t)NN * NN, sizeof(int));
    s->hb_sum_opp = (double *)calloc(NN, sizeof(double));
    int kmax = NN > np ? NN : np;
    int *small = (int *)malloc(sizeof(int) * kmax);
    int *large = (int *)malloc(sizeof(int) * kmax);
    double *scaled = (double *)malloc(sizeof(double) * kmax);
    int ij = 0;
    for (int I = 0; I < N; ++I)
        for (int J = I + 1; J < N; ++J, ++ij) {
            double sum = 0.0;
            double *w = s->hb_w_same + (size_t)ij * np;
            int ab = 0;
            for (int A = 0; A < N; ++A)
                for (int B = A + 1; B < N; ++B, ++ab) {
                    double v = eri(s, A, I, B, J) - eri(s, A, J, B, I);
                    double x = fabs(v);
                    if (A == I || A == J || B == I || B == J) x = 0.0;
                    w[ab] = x;
                    sum = sum + x;
                }
            s->hb_sum_same[ij] = sum;
            alias_build(w, np, sum, s->hb_p_same + (size_t)ij * np, s->hb_a_same + (size_t)ij * np,
                        small, large, scaled);
        }
    for (int I = 0; I < N; ++I)
        for (int J = 0; J < N; ++J) {
            double sum = 0.0;
            double *w = s->hb_w_opp + (size_t)(I * N + J) * NN;
            for (int A = 0; A < N; ++A)
                for (int B = 0; B < N; ++B) {
                    double x = fabs(eri(s, A, I, B, J));
                    if (A == I || B == J) x = 0.0;
                    w[A * N + B] = x;
                    sum = sum + x;
                }
            s->hb_sum_opp[I * N + J] = sum;
            alias_build(w, NN, sum, s->hb_p_opp + (size_t)(I * N + J) * NN,
                        s->hb_a_opp + (size_t)(I * N + J) * NN, small, large, scaled);
        }
    free(small); free(large); free(scaled);
}

/* Alias draw from one 64-bit word x: column c = floor(x K / 2^64), uniform
 * over the K columns; the coin is the fraction this leaves, the low 64 bits
 * of x K taken as a 53-bit uniform (for fixed c they run over a grid of step
 * K / 2^64 covering [0, 1), so the coin is uniform and independent of c to
 * that resolution).  Column c is kept with probability prob_c, else the
 * draw goes to alias_c. */
static int alias_draw(const double *prob, const int *alias, int K, uint64_t xc)
{
    int c = (int)pick(xc, (uint64_t)K);
    uint64_t frac = xc * (uint64_t)K;
    double coin = unif(frac);
    return coin < prob[c] ? c : alias[c];
}

int orc_pchb_gen(const orc_sys *s, det_t d, const uint64_t r1[4],
                 double p_single, double p_opp, det_t *tgt, double *pgen)
{
    int N = s->N;
    int n = s->na + s->nb;
    double u0 = unif(r1[0]);
    if (u0 < p_single) {
        uint64_t idx1 = pick(r1[1], (uint64_t)n);
        uint64_t c2 = orc_uniform_count2(s, d, 1, idx1);
        if (c2 == 0) return 0;
        return orc_uniform_apply(s, d, 1, idx1, pick(r1[2], c2), p_single, tgt, pgen);
    }
    int occa[64], occb[64], na = 0, nb = 0;
    for (int p = 0; p < N; ++p) {
        if ((d.a >> p) & 1) occa[na++] = p;
        if ((d.b >> p) & 1) occb[nb++] = p;
    }
    uint64_t n_opp = (uint64_t)na * (uint64_t)nb;
    uint64_t npa = (uint64_t)na * (uint64_t)(na - (na > 0)) / 2;
    uint64_t npb = (uint64_t)nb * (uint64_t)(nb - (nb > 0)) / 2;
    uint64_t n_same = npa + npb;
    double pd = 1.0 - p_single;
    /* the pair class from the same uniform: beyond p_single the first
     * p_double p_opp of it is the opposite-spin class */
    double pdo = pd * p_opp;
    double thr = p_single + pdo;
    int opp = u0 < thr;
    if (opp) {
        if (n_opp == 0) return 0;
        uint64_t q = pick(r1[1], n_opp);
        int I = occa[q / (uint64_t)nb], J = occb[q % (uint64_t)nb];
        double sum = s->hb_sum_opp[I * N + J];
        if (sum == 0.0) return 0;
        size_t row = (size_t)(I * N + J) * N * N;
        int c = alias_draw(s->hb_p_opp + row, s->hb_a_opp + row, N * N, r1[2]);
        double wc = s->hb_w_opp[row + c];
        if (wc == 0.0) return 0;
        int A = c / N, B = c % N;
        if (((d.a >> A) & 1) || ((d.b >> B) & 1)) return 0;
        det_t t = d;
        t.a &= ~(1ULL << I); t.b &= ~(1ULL << J); t.a |= 1ULL << A; t.b |= 1ULL << B;
        *tgt = t;
        double p1 = pd * p_opp;
        double p2 = p1 / (double)n_opp;
        double pab = wc / sum;
        *pgen = p2 * pab;
        return 1;
    }
    if (n_same == 0) return 0;
    uint64_t q = pick(r1[1], n_same);
    int sig = q >= npa;
    if (sig) q -= npa;
    const int *occ = sig ? occb : occa;
    int no = sig ? nb : na;
    int e1 = -1, e2 = -1;
    uint64_t cc = 0;
    for (int x = 0; x < no && e1 < 0; ++x)
        for (int y = x + 1; y < no; ++y) {
            if (cc == q) { e1 = x; e2 = y; break; }
            cc++;
        }
    int I = occ[e1], J = occ[e2];
    int np = N * (N - 1) / 2;
    int ij = I * (2 * N - I - 1) / 2 + (J - I - 1);
    double sum = s->hb_sum_same[ij];
    if (sum == 0.0) return 0;
    size_t row = (size_t)ij * np;
    int c = alias_draw(s->hb_p_same + row, s->hb_a_same + row, np, r1[2]);
    double wc = s->hb_w_same[row + c];
    if (wc == 0.0) return 0;
    int A = -1, B = -1, cnt = 0;
    for (int x = 0; x < N && A < 0; ++x)
        for (int y = x + 1; y < N; ++y) {
            if (cnt == c) { A = x; B = y; break; }
            cnt++;
        }
    uint64_t mask = sig ? d.b : d.a;
    if (((mask >> A) & 1) || ((mask >> B) & 1)) return 0;
    mask &= ~(1ULL << I); mask &= ~(1ULL << J); mask |= 1ULL << A; mask |= 1ULL << B;
    det_t t = d;
    if (sig) t.b = mask; else t.a = mask;
    *tgt = t;
    double p1 = pd * (1.0 - p_opp);
    double p2 = p1 / (double)n_same;
    double pab = wc / sum;
    *pgen = p2 * pab;
    return 1;
}

/* Alias-table access for the reconstruction test: row of class `opp`. */
void orc_pchb_row(const orc_sys *s, int opp, int row, double *w, double *prob, int *alias,
                  double *sum)
{
    int N = s->N;
    int K = opp ? N * N : N * (N - 1) / 2;
    const double *W = opp ? s->hb_w_opp : s->hb_w_same;
    const double *P = opp ? s->hb_p_opp : s->hb_p_same;
    const int *A = opp ? s->hb_a_opp : s->hb_a_same;
    for (int c = 0; c < K; ++c) {
        w[c] = W[(size_t)row * K + c];
        prob[c] = P[(size_t)row * K + c];
        alias[c] = A[(size_t)row * K + c];
    }
    *sum = opp ? s->hb_sum_opp[row] : s->hb_sum_same[row];
}

/* ------------------------------------------------------------------------- */
/* On-the-fly Cauchy-Schwarz (CS) and Part-Exact (PE) generators              */
/* (Appendix A.2).  No tables: every draw builds its cumulative probability  */
/* functions (CPFs) from the integrals.                                        */
/*                                                                             */
/* Singles (weighted, Appendix A.2 "Single excitations"): electron i uniform  */
/* among the n; hole a among the same-spin holes with weight |<D_i^a|H|D>|.   */
/*   p_gen = (p_single / n) (w_a / sum_h w_h).                                 */
/* Doubles, electron pair: i uniform among the n; j != i from the CPF with    */
/* weights |<ik|ik>| = |(ii|kk)| times p_opp (opposite spins) or 1 - p_opp    */
/* (equal spins).  p(ij) = (w_ij / S_i + w_ji / S_j) / n, where S_x is the    */
/* sum of the CPF built from electron x.                                       */
/*   Readings: the paper writes 1/N in p(ij), but i is drawn among the n      */
/*   electrons, so the factor is 1/n; the two printed forms F_{j-i} and        */
/*   F_{j-1} of the CPF increment are read as F_{j-1}, the weight of j.       */
/* Opposite spins (i beta, j alpha by the paper's convention): hole a among   */
/* the beta holes with weight sqrt(<aa|ii>) = sqrt((ia|ia)); hole b among the */
/* alpha holes with weight sqrt(|<ij|ab>|) = sqrt(|(ia|jb)|) (PE) or          */
/* sqrt(<bb|jj>) (CS).  p_gen = p_double p(ij) p(a|i) p(b|ija).               */
/* Equal spins sigma: hole a among the sigma holes with weight                */
/* sqrt(<aa|ii>) + sqrt(<aa|jj>); hole b among the other sigma holes with     */
/* weight sqrt(|<ij|ab> - <ij|ba>|) = sqrt(|(ia|jb) - (ib|ja)|) (PE) or the    */
/* first-hole weight (CS).  Either order of the holes gives the same target: */
/*   p_gen = p_double p(ij) [p(a|ij) p(b|ija) + p(b|ij) p(a|ijb)].            */
/* Readings: there are no point-group labels, so every orbital shares one     */
/* irrep and the symmetry restriction of the paper is void; Coulomb integrals */
/* and the arguments of the square roots enter as |x|: the same for physical */
/* integrals, and a valid CPF for model integrals where (ii|kk) may be < 0.  */
/*                                                                             */
/* CPF inversion: xi = u * F_last with u uniform in [0, 1); the chosen index   */
/* is the first k with F_k > xi, i.e. F_{k-1} <= xi < F_k (Reading: the       */
/* half-open form never selects a zero weight).  If rounding leaves no such  */
/* k, the last index of positive weight is taken.  A CPF whose last value is  */
/* zero makes the draw null.  F is summed in the order of the candidates     */
/* (ascending orbitals, alpha before beta).                                   */
/* Random lanes: block SPAWN [0] single/double, [1] first electron, [2]       */
/* second electron (doubles) or the hole (singles), [3] acceptance; block     */
/* SPAWN2 [0] first hole, [1] second hole.                                    */
/* ------------------------------------------------------------------------- */

static double sqrt_abs(double x) { return sqrt(fabs(x)); }

/* Index into w[0..m) by CPF inversion with uniform u; -1 if all weights are 0. */
static int cpf_invert(const double *w, int m, double u, double *total)
{
    double sum = 0.0;
    for (int k = 0; k < m; ++k) sum = sum + w[k];
    *total = sum;
    if (sum == 0.0) return -1;
    double xi = u * sum;
    double F = 0.0;
    int last = -1;
    for (int k = 0; k < m; ++k) {
        F = F + w[k];
        if (w[k] > 0.0) last = k;
        if (F > xi) return k;
    }
    return last;
}

static double sum_of(const double *w, int m)
{
    double s = 0.0;
    for (int k = 0; k < m; ++k) s = s + w[k];
    return s;
}

/* Electron-pair CPF weights of electron x over the occupied list occ[0..n). */
static void pair_weights(const orc_sys *s, const int *occ, int n, int x, double p_opp, double *w)
{
    double q_same = 1.0 - p_opp;
    int px = so_orb(s, occ[x]);
    for (int k = 0; k < n; ++k) {
        if (k == x) { w[k] = 0.0; continue; }
        int pk = so_orb(s, occ[k]);
        double bias = so_spin(s, occ[k]) != so_spin(s, occ[x]) ? p_opp : q_same;
        w[k] = fabs(eri(s, px, px, pk, pk)) * bias;
    }
}

int orc_cs_gen(const orc_sys *s, det_t d, const uint64_t r1[4], const uint64_t r2[4],
               double p_single, double p_opp, int exact, det_t *tgt, double *pgen)
{
    int occ[128], hol[64];
    double w[128], w2[128], wr[128];
    int n = det_occ_list(s, d, occ);
    if (unif(r1[0]) < p_single) {
        int e = (int)pick(r1[1], (uint64_t)n);
        int i = occ[e];
        int h = holes_of_spin(s, d, so_spin(s, i), hol);
        for (int x = 0; x < h; ++x) w[x] = fabs(hsingle(s, d, i, hol[x]));
        double tot;
        int x = cpf_invert(w, h, unif(r1[2]), &tot);
        if (x < 0) return 0;
        det_t t = d; det_set(s, &t, i, 0); det_set(s, &t, hol[x], 1);
        *tgt = t;
        double pi = p_single / (double)n;
        double pa = w[x] / tot;
        *pgen = pi * pa;
        return 1;
    }
    if (n < 2) return 0;
    double pd = 1.0 - p_single;
    /* electron pair */
    int e1 = (int)pick(r1[1], (uint64_t)n);
    pair_weights(s, occ, n, e1, p_opp, w);
    double S1;
    int e2 = cpf_invert(w, n, unif(r1[2]), &S1);
    if (e2 < 0) return 0;
    pair_weights(s, occ, n, e2, p_opp, w2);
    double S2 = sum_of(w2, n);
    double pij = (w[e2] / S1 + w2[e1] / S2) / (double)n;
    int i = occ[e1], j = occ[e2];
    if (i > j) { int tmp = i; i = j; j = tmp; }  /* canonical order */
    int pi_ = so_orb(s, i), pj_ = so_orb(s, j);
    det_t t = d;
    if (so_spin(s, i) != so_spin(s, j)) {
        /* i alpha (pi_), j beta (pj_): first hole beta, from electron j */
        int hb[64], ha[64];
        int nhb = holes_of_spin(s, d, 1, hb);
        int nha = holes_of_spin(s, d, 0, ha);
        for (int x = 0; x < nhb; ++x) w[x] = sqrt_abs(eri(s, pj_, so_orb(s, hb[x]), so_orb(s, hb[x]), pj_));
        double SA;
        int xa = cpf_invert(w, nhb, unif(r2[0]), &SA);
        if (xa < 0) return 0;
        int A = so_orb(s, hb[xa]);
        for (int x = 0; x < nha; ++x) {
            int B = so_orb(s, ha[x]);
            if (exact) w2[x] = sqrt_abs(eri(s, pj_, A, pi_, B));
            else w2[x] = sqrt_abs(eri(s, pi_, B, B, pi_));
        }
        double SB;
        int xb = cpf_invert(w2, nha, unif(r2[1]), &SB);
        if (xb < 0) return 0;
        double p1 = pd * pij;
        double p2 = p1 * (w[xa] / SA);
        *pgen = p2 * (w2[xb] / SB);
        det_set(s, &t, i, 0); det_set(s, &t, j, 0);
        det_set(s, &t, ha[xb], 1); det_set(s, &t, hb[xa], 1);
        *tgt = t;
        return 1;
    }
    int sig = so_spin(s, i);
    int h = holes_of_spin(s, d, sig, hol);
    for (int x = 0; x < h; ++x) {
        int P = so_orb(s, hol[x]);
        double ci = sqrt_abs(eri(s, pi_, P, P, pi_));
        double cj = sqrt_abs(eri(s, pj_, P, P, pj_));
        w[x] = ci + cj;
    }
    double SA;
    int xa = cpf_invert(w, h, unif(r2[0]), &SA);
    if (xa < 0) return 0;
    int A = so_orb(s, hol[xa]);
    for (int x = 0; x < h; ++x) {
        int P = so_orb(s, hol[x]);
        if (x == xa) { w2[x] = 0.0; continue; }
        if (exact) {
            double dir = eri(s, pi_, A, pj_, P);
            double exc = eri(s, pi_, P, pj_, A);
            w2[x] = sqrt_abs(dir - exc);
        } else {
            w2[x] = w[x];
        }
    }
    double SB;
    int xb = cpf_invert(w2, h, unif(r2[1]), &SB);
    if (xb < 0) return 0;
    /* the reverse order: b first, then a */
    int Bo = so_orb(s, hol[xb]);
    for (int x = 0; x < h; ++x) {
        int P = so_orb(s, hol[x]);
        if (x == xb) { wr[x] = 0.0; continue; }
        if (exact) {
            double dir = eri(s, pi_, Bo, pj_, P);
            double exc = eri(s, pi_, P, pj_, Bo);
            wr[x] = sqrt_abs(dir - exc);
        } else {
            wr[x] = w[x];
        }
    }
    double SR = sum_of(wr, h);
    double pab = (w[xa] / SA) * (w2[xb] / SB);
    double pba = (w[xb] / SA) * (wr[xa] / SR);
    double p1 = pd * pij;
    *pgen = p1 * (pab + pba);
    det_set(s, &t, i, 0); det_set(s, &t, j, 0);
    det_set(s, &t, hol[xa], 1); det_set(s, &t, hol[xb], 1);
    *tgt = t;
    return 1;
}

/* ------------------------------------------------------------------------- */
/* Flat entry points for the Python wrapper (dets as alpha/beta mask pairs).  */
/* ------------------------------------------------------------------------- */
double orc_hdiag(const orc_sys *s, uint64_t a, uint64_t b)
{
    det_t d = {a, b};
    return orc_hdiag_det(s, d);
}

double orc_hij(const orc_sys *s, uint64_t a1, uint64_t b1, uint64_t a2, uint64_t b2)
{
    det_t d1 = {a1, b1}, d2 = {a2, b2};
    return orc_hij_det(s, d1, d2);
}

/* One row of the deterministic-space matrix, as orc_run_set_core fills it:
 * out[j] = <D_row|H|D_j> = orc_hij(D_j, D_row) for the n determinants
 * (a[j], b[j]) (out[j] = 0 where D_j = D_row). */
void orc_hij_row(const orc_sys *s, uint64_t ar, uint64_t br, const uint64_t *a, const uint64_t *b, int64_t n,
                 double *out)
{
    det_t dr = {ar, br};
    for (int64_t j = 0; j < n; ++j) {
        det_t dj = {a[j], b[j]};
        out[j] = (a[j] == ar && b[j] == br) ? 0.0 : orc_hij_det(s, dj, dr);
    }
}

/* Draw-level generator entry (for frequency tests): returns 1 and the target
 * for a null-free draw from the Philox block of (det, t, k). */
int orc_generate(const orc_run *r, uint64_t a, uint64_t b, int64_t t, uint64_t k,
                 uint64_t *ta, uint64_t *tb, double *pgen, double *H)
{
    det_t d = {a, b}, tgt;
    uint64_t rr[4];
    spawn_words(r, d, t, k, rr);
    int ok;
    if (r->p.gen == GEN_UNIFORM) ok = gen_uniform(r->s, d, rr, r->p.p_single, &tgt, pgen);
    else if (r->p.gen == GEN_LATTICE) ok = gen_lattice(r->s, d, rr, &tgt, pgen);
    else if (r->p.gen == GEN_PCHB) ok = orc_pchb_gen(r->s, d, rr, r->p.p_single, r->p.p_opp, &tgt, pgen);
    else {
        uint64_t r2[4] = {0, 0, 0, 0};
        draw_block(r, d, t, k, PURPOSE_SPAWN2, r2);  /* words 0-1 */
        ok = orc_cs_gen(r->s, d, rr, r2, r->p.p_single, r->p.p_opp, r->p.gen == GEN_PE, &tgt, pgen);
    }
    if (!ok) return 0;
    *ta = tgt.a; *tb = tgt.b;
    *H = orc_hij_det(r->s, d, tgt);
    return 1;
}

int orc_uniform_apply_flat(const orc_sys *s, uint64_t a, uint64_t b, int single, uint64_t idx1,
                           uint64_t idx2, double p_single, uint64_t *ta, uint64_t *tb, double *pgen)
{
    det_t d = {a, b}, t;
    int ok = orc_uniform_apply(s, d, single, idx1, idx2, p_single, &t, pgen);
    if (ok) { *ta = t.a; *tb = t.b; }
    return ok;
}

uint64_t orc_uniform_count2_flat(const orc_sys *s, uint64_t a, uint64_t b, int single, uint64_t idx1)
{
    det_t d = {a, b};
    return orc_uniform_count2(s, d, single, idx1);
}

int orc_lattice_apply_flat(const orc_sys *s, uint64_t a, uint64_t b, uint64_t idx1, uint64_t idx2,
                           uint64_t *ta, uint64_t *tb, double *pgen)
{
    det_t d = {a, b}, t;
    int ok = orc_lattice_apply(s, d, idx1, idx2, &t, pgen);
    if (ok) { *ta = t.a; *tb = t.b; }
    return ok;
}

/* Estimators of the current population (Sec. IV, Eq. (proje)): N_w = sum |C_i|, C_ref and sum_{j != ref} H_ref,j C_j. */
void orc_run_estimate(const orc_run *r, double *nw_out, double *nref_out, double *enum_out)
{
    double nw = 0.0, nref = 0.0, en = 0.0;
    for (int64_t x = 0; x < r->n; ++x) {
        const ent_t *e = &r->list[x];
        nw = nw + fabs(e->v);
        if (det_eq(e->d, r->proj)) { nref = e->v; continue; }
        int lvl = __builtin_popcountll(e->d.a ^ r->proj.a) + __builtin_popcountll(e->d.b ^ r->proj.b);
        if (lvl == 2 || lvl == 4) {
            double h = orc_hij_det(r->s, r->proj, e->d);
            double c = h * e->v;
            en = en + c;
        }
    }
    *nw_out = nw; *nref_out = nref; *enum_out = en;
}

void orc_layout(const orc_sys *s, uint64_t a, uint64_t b, uint64_t *w0, uint64_t *w1)
{
    det_t d = {a, b};
    layout_words(s, d, w0, w1);
}

void orc_unlayout(const orc_sys *s, uint64_t w0, uint64_t w1, uint64_t *a, uint64_t *b)
{
    det_t d = from_layout(s, w0, w1);
    *a = d.a; *b = d.b;
}
