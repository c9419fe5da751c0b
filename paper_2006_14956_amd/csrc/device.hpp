// Device building blocks of the FCIQMC step for CDNA4 (gfx950, wave64).
//
// Determinant layouts (W = 64-bit words per determinant):
//   W = 1 (N <= 32): alpha orbital p at bit p, beta orbital p at bit 32 + p;
//   W = 2 (N <= 63): word 0 = alpha mask, word 1 = beta mask.
// In both, bit order equals the canonical spin-orbital order (all alpha
// orbitals, then all beta orbitals), which fixes the fermionic signs.
//
// Floating point: every expression is written as the sequence of IEEE
// binary64 operations it stands for; the library is built with
// -ffp-contract=off so no multiply-add is fused.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fq {

constexpr uint64_t kEmpty = ~0ULL;       // unused hash slot
constexpr uint64_t kLocked = ~0ULL - 1;  // slot being claimed (2-word keys only)

// Purposes of random blocks (part of the Philox key; the second block of a
// four-word draw uses purpose + 128).
enum : uint64_t { kSpawn = 0, kSpawn2 = 1, kDeath = 2, kAnn = 4 };

// Error / overflow flags raised on the device, read back by the host.
enum : unsigned { kFlagSpawnCap = 1u, kFlagTable = 2u, kFlagStore = 4u, kFlagBloom = 8u,
                  kFlagSpin = 16u, kFlagPop = 32u };

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64
// multiplies with a Weyl-sequence key schedule.  The 32-bit form suits this
// target (a 32x32 product is one instruction pair; a 64x64 product is four
// 64-bit multiply-adds).
// --------------------------------------------------------------------------
struct R4 { uint64_t x[4]; };
struct R2 { uint64_t x[2]; };

__device__ __forceinline__ R2 philox4x32(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                         uint32_t k1) {
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    // rounds kept as a loop: the key schedule then stays two scalar adds per
    // round instead of twenty hoisted round keys per stream spilled to
    // vector lanes.  Two rounds per pass, so that the words land back in
    // their own registers without moves.  Each product is formed as one
    // 32x32 -> 64-bit multiply (one v_mad_u64_u32 gives both halves, where a
    // separate high and low product take two quarter-rate instructions).
#pragma unroll 1
    for (int r = 0; r < 5; ++r) {
        const uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
        const uint32_t a0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, a1 = (uint32_t)p1;
        const uint32_t a2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1, a3 = (uint32_t)p0;
        k0 += W0; k1 += W1;
        const uint64_t q0 = (uint64_t)M0 * a0, q1 = (uint64_t)M1 * a2;
        c0 = (uint32_t)(q1 >> 32) ^ a1 ^ k0; c1 = (uint32_t)q1;
        c2 = (uint32_t)(q0 >> 32) ^ a3 ^ k1; c3 = (uint32_t)q0;
        k0 += W0; k1 += W1;
    }
    R2 o;
    o.x[0] = (uint64_t)c0 | ((uint64_t)c1 << 32);
    o.x[1] = (uint64_t)c2 | ((uint64_t)c3 << 32);
    return o;
}

// Choice in [0, m): floor(x m / 2^64).
__device__ __forceinline__ uint64_t pick(uint64_t x, uint64_t m) { return __umul64hi(x, m); }
// Choice in [0, m) from a 32-bit word: floor(x m / 2^32).
__device__ __forceinline__ uint32_t pick32(uint32_t x, uint32_t m) { return __umulhi(x, m); }
// Uniform in [0,1) from the top 53 bits.
__device__ __forceinline__ double unif(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

// --------------------------------------------------------------------------
// Determinant keys.
// --------------------------------------------------------------------------
template <int W> struct Key { uint64_t w[W]; };

template <int W> __device__ __forceinline__ uint64_t key_alpha(const Key<W>& k) {
    if constexpr (W == 1) return k.w[0] & 0xFFFFFFFFULL; else return k.w[0];
}
template <int W> __device__ __forceinline__ uint64_t key_beta(const Key<W>& k) {
    if constexpr (W == 1) return k.w[0] >> 32; else return k.w[1];
}
template <int W> __device__ __forceinline__ Key<W> make_key(uint64_t a, uint64_t b) {
    Key<W> k;
    if constexpr (W == 1) { k.w[0] = a | (b << 32); } else { k.w[0] = a; k.w[1] = b; }
    return k;
}
template <int W> __device__ __forceinline__ bool key_eq(const Key<W>& x, const Key<W>& y) {
    if constexpr (W == 1) return x.w[0] == y.w[0]; else return x.w[0] == y.w[0] && x.w[1] == y.w[1];
}
template <int W> __device__ __forceinline__ Key<W> load_key(const uint64_t* p) {
    Key<W> k;
    if constexpr (W == 1) { k.w[0] = p[0]; }
    else { const ulonglong2 v = *reinterpret_cast<const ulonglong2*>(p); k.w[0] = v.x; k.w[1] = v.y; }
    return k;
}
template <int W> __device__ __forceinline__ void store_key(uint64_t* p, const Key<W>& k) {
    if constexpr (W == 1) { p[0] = k.w[0]; }
    else { ulonglong2 v; v.x = k.w[0]; v.y = k.w[1]; *reinterpret_cast<ulonglong2*>(p) = v; }
}

// splitmix64 finaliser (a bijection of 64-bit words); partitions
// determinants into buckets (high bits), places them in the per-bucket LDS
// table (low bits) and hashes the identities of random streams.
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    x ^= x >> 30; x *= 0xBF58476D1CE4E5B9ULL;
    x ^= x >> 27; x *= 0x94D049BB133111EBULL;
    x ^= x >> 31;
    return x;
}

// Random words of (determinant, iteration, ordinal, purpose): a Philox
// block with counter (64-bit identity of the determinant, low 32 bits of t
// and of the ordinal) and key = mix(mix(seed) ^ (replica << 8 | purpose)).
// A one-word determinant is its own identity; a two-word one is hashed
// (mix(w0 ^ mix(w1 + c))).  draw2 gives the block's two 64-bit words; draw
// gives four, the second pair from the block of purpose + 128.
template <int W> __device__ __forceinline__ R2 draw2(const Key<W>& k, int64_t t, uint64_t ord,
                                                     uint64_t purpose, uint64_t seed, uint64_t rep) {
    const uint64_t id = W == 1 ? k.w[0] : mix64(k.w[0] ^ mix64(k.w[W - 1] + 0x632BE59BD9B4E019ULL));
    const uint64_t sk = mix64(mix64(seed) ^ ((rep << 8) | purpose));
    return philox4x32((uint32_t)id, (uint32_t)(id >> 32), (uint32_t)t, (uint32_t)ord, (uint32_t)sk,
                      (uint32_t)(sk >> 32));
}
template <int W> __device__ __forceinline__ R4 draw(const Key<W>& k, int64_t t, uint64_t ord,
                                                    uint64_t purpose, uint64_t seed, uint64_t rep) {
    const R2 a = draw2<W>(k, t, ord, purpose, seed, rep);
    const R2 b = draw2<W>(k, t, ord, purpose | 128, seed, rep);
    R4 o;
    o.x[0] = a.x[0]; o.x[1] = a.x[1]; o.x[2] = b.x[0]; o.x[3] = b.x[1];
    return o;
}

template <int W> __device__ __forceinline__ uint64_t key_hash(const Key<W>& k) {
    if constexpr (W == 1) return mix64(k.w[0] + 0x632BE59BD9B4E019ULL);
    else return mix64(k.w[0] ^ mix64(k.w[1] + 0x632BE59BD9B4E019ULL));
}
__device__ __forceinline__ uint32_t bucket_of(uint64_t h, uint32_t B) { return (uint32_t)__umul64hi(h, B); }

// --------------------------------------------------------------------------
// Bit helpers.
// --------------------------------------------------------------------------
__device__ __forceinline__ int ctz64(uint64_t x) { return __builtin_ctzll(x); }
__device__ __forceinline__ int popc64(uint64_t x) { return __popcll(x); }
__device__ __forceinline__ uint64_t low_mask(int p) { return (1ULL << p) - 1ULL; }

// Position of the k-th (0-based) set bit of x; x must have more than k bits set.
__device__ __forceinline__ int select64(uint64_t x, int k) {
    int pos = 0;
    int c = __popc((uint32_t)x);
    if (k >= c) { k -= c; x >>= 32; pos = 32; }
    uint32_t w = (uint32_t)x;
    c = __popc(w & 0xFFFFu); if (k >= c) { k -= c; w >>= 16; pos += 16; }
    c = __popc(w & 0xFFu);   if (k >= c) { k -= c; w >>= 8;  pos += 8; }
    c = __popc(w & 0xFu);    if (k >= c) { k -= c; w >>= 4;  pos += 4; }
    c = __popc(w & 0x3u);    if (k >= c) { k -= c; w >>= 2;  pos += 2; }
    c = (int)(w & 1u);       if (k >= c) { pos += 1; }
    return pos;
}

// Occupied spin orbitals below (spin s, orbital p) in canonical order.
__device__ __forceinline__ int below(uint64_t A, uint64_t B, int s, int p) {
    return s == 0 ? popc64(A & low_mask(p)) : popc64(A) + popc64(B & low_mask(p));
}
__device__ __forceinline__ void clear_so(uint64_t& A, uint64_t& B, int s, int p) {
    if (s == 0) A &= ~(1ULL << p); else B &= ~(1ULL << p);
}
__device__ __forceinline__ void set_so(uint64_t& A, uint64_t& B, int s, int p) {
    if (s == 0) A |= (1ULL << p); else B |= (1ULL << p);
}

// Decode a lexicographic pair index q over C(n,2) pairs (x<y) of n items
// (n <= 128): x is the last row whose first index off(x) = x(2n-x-1)/2 is
// <= q, from the quadratic's root in single precision, then set exactly by
// comparing with off(x) and off(x+1).
__device__ __forceinline__ void pair_decode(uint64_t q64, int n, int& x, int& y) {
    const int q = (int)q64;
    const int m = 2 * n - 1;
    int e = (int)(((float)m - sqrtf((float)(m * m - 8 * q))) * 0.5f);
    e = e < 0 ? 0 : (e > n - 2 ? n - 2 : e);
    if (e * (m - e) / 2 > q) --e;
    if ((e + 1) * (m - e - 1) / 2 <= q) ++e;
    x = e;
    y = e + 1 + (q - e * (m - e) / 2);
}

// floor(q / d) for q < 4096 and 1 <= d <= 64 from m = ceil(2^20 / d): exact,
// since q d < 2^20, and q m < 2^32 (Granlund and Montgomery's division by
// invariant integers; the pair and column indices of N <= 64 orbitals).
__device__ __forceinline__ uint32_t div_small(uint32_t q, uint32_t m) { return (q * m) >> 20; }

// --------------------------------------------------------------------------
// Integrals.
// --------------------------------------------------------------------------
// One column of a heat-bath alias table, one 8-byte word: the alias
// threshold prob (in [0, 1]) as T = floor(prob 2^48) in bits 15..63 and the
// column's alias in bits 0..14.  A draw's 53-bit coin f (the table is taken
// when f < prob 2^53) is decided by its top 48 bits against T; only when
// those equal T (probability 2^-48) does the draw read the exact FP64
// threshold, kept beside the table.  The drawn column's signed two-electron
// value v (whose magnitude is its weight) comes from the packed integrals,
// a table small enough to stay in L2.  The rows a population draws from
// most (pairs of the orbitals most determinants occupy) then take a few MB.
constexpr int kHbAliasBits = 15;
__host__ __device__ __forceinline__ uint64_t hb_pack(double prob, int alias) {
    return ((uint64_t)(prob * 0x1p48) << kHbAliasBits) | (uint64_t)alias;
}

struct SysView {
    int N, na, nb, n;
    int onsite;           // two-electron integrals vanish except (pp|pp)
    const double* h1;     // N*N
    const double* eri;    // 8-fold packed
    const double* J;      // J[p*N+q] = (pp|qq)
    const double* K;      // K[p*N+q] = (pq|qp)
    const double* X;      // X[p*N+q] = (pp|qq) - (pq|qp), the same-spin pair term
    const double* Hd;     // Hd[p] = h_pp
    const double* U;      // U[p] = (pp|pp)
    const int* deg;       // lattice degree
    const int* nbr;       // N*N ascending neighbour lists
    // exact probabilities of the lattice generator's 32-bit choices:
    // lat_pe[e] of electron e among the n, lat_pz[z*N + d] of neighbour d
    // among z (the share of 32-bit words x with floor(x m / 2^32) = index)
    const double* lat_pe;
    const double* lat_pz;
    // pre-computed heat-bath tables (see the PCHB generator)
    const double* SK;     // SK[p*N+q] = sqrt(|(pq|qp)|), the Cauchy-Schwarz hole weights
    const uint64_t* hb_opp;   // rows (I alpha, J beta), N^2 columns each
    const uint64_t* hb_same;  // rows I < J, N(N-1)/2 columns each
    const double* hbp_opp;    // their exact alias thresholds, same layout
    const double* hbp_same;
    const double* hb_sum_opp;   // row sums of the weights
    const double* hb_sum_same;
    const int* pair_of;   // same-spin column index -> A*64+B
    uint32_t mN, mnb;     // ceil(2^20 / N), ceil(2^20 / nb) (0 for nb = 0): div_small multipliers
};

__device__ __forceinline__ int tri(int p, int q) { return p >= q ? p * (p + 1) / 2 + q : q * (q + 1) / 2 + p; }
__device__ __forceinline__ double eri(const SysView& s, int p, int q, int r, int t) {
    const int P = tri(p, q), Q = tri(r, t);
    return s.eri[tri(P, Q)];
}

// <D_j|H|D_i>, D_j = sgn a+_a a_i D_i, electron (sg, pi) -> hole (sg, pa).
// Sum over the other electrons of D_i in canonical order.
__device__ __forceinline__ double h_single(const SysView& s, uint64_t a, uint64_t b, int sg, int pi,
                                           int pa) {
    const int N = s.N;
    double v = s.h1[pi * N + pa];
    if (!s.onsite) {
        for (uint64_t x = a; x; x &= x - 1) {
            const int k = ctz64(x);
            if (sg == 0 && k == pi) continue;
            const double d = eri(s, pi, pa, k, k);
            if (sg == 0) { const double e = eri(s, pi, k, k, pa); const double t = d - e; v = v + t; }
            else v = v + d;
        }
        for (uint64_t x = b; x; x &= x - 1) {
            const int k = ctz64(x);
            if (sg == 1 && k == pi) continue;
            const double d = eri(s, pi, pa, k, k);
            if (sg == 1) { const double e = eri(s, pi, k, k, pa); const double t = d - e; v = v + t; }
            else v = v + d;
        }
    }
    uint64_t A = a, B = b;
    int par = below(A, B, sg, pi);
    clear_so(A, B, sg, pi);
    par += below(A, B, sg, pa);
    return (par & 1) ? -v : v;
}

// <D_j|H|D_i>, D_j = sgn a+_a a+_b a_j a_i D_i with i<j and a<b canonical;
// the operator's coefficient is <ab||ij> = (ai|bj) - (aj|bi) on matching spins.
// Fermion sign of a+_a a+_b a_j a_i applied to (a, b): 1 if odd.
__device__ __forceinline__ int double_parity(uint64_t a, uint64_t b, int si, int pi, int sj, int pj, int sa,
                                             int pa, int sb, int pb) {
    uint64_t A = a, B = b;
    int par = below(A, B, si, pi);
    clear_so(A, B, si, pi);
    par += below(A, B, sj, pj);
    clear_so(A, B, sj, pj);
    par += below(A, B, sb, pb);
    set_so(A, B, sb, pb);
    par += below(A, B, sa, pa);
    return par & 1;
}

// The same sign where A takes the spin of I and B that of J (the heat-bath
// draw), 1 if odd.  a_I passes a_J and a+_B (B is empty, so B != I), which
// makes the operator (a+_A a_I)(a+_B a_J): the move J -> B on D_i, then
// I -> A on what it leaves.  A move p -> h inside one spin string w flips
// the sign once per occupied orbital strictly between p and h;
// popc(w & (low(p) ^ low(h))) counts those and, when p < h, p itself.  The
// second move sees J gone and B present, which changes its count only
// where both pairs share a spin and J or B lies between I and A.  Equal to
// double_parity(a, b, sI, I, sJ, J, sI, A, sJ, B) for every valid move.
__device__ __forceinline__ int move_pair_parity(uint64_t a, uint64_t b, int sI, int I, int sJ, int J, int A,
                                                int B) {
    const uint64_t mI = low_mask(I) ^ low_mask(A);
    const uint64_t mJ = low_mask(J) ^ low_mask(B);
    const uint64_t wI = sI ? b : a, wJ = sJ ? b : a;
    int par = popc64((wI & mI) ^ (wJ & mJ)) + (I < A ? 1 : 0) + (J < B ? 1 : 0);
    if (sI == sJ) par += (int)(((mI >> J) ^ (mI >> B)) & 1ULL);
    return par & 1;
}

__device__ __forceinline__ double h_double(const SysView& s, uint64_t a, uint64_t b, int si, int pi,
                                           int sj, int pj, int sa, int pa, int sb, int pb) {
    const double direct = (sa == si && sb == sj) ? eri(s, pa, pi, pb, pj) : 0.0;
    const double exch = (sa == sj && sb == si) ? eri(s, pa, pj, pb, pi) : 0.0;
    double v;
    if (si == sj) v = direct - exch;
    else v = (sa == si) ? direct : -exch;
    return double_parity(a, b, si, pi, sj, pj, sa, pa, sb, pb) ? -v : v;
}

// H_ii: sum_p h_pp + sum_{p<q} [(pp|qq) - delta(spin)(pq|qp)], canonical order,
// from tables hd[p] = h_pp, X[p*N+q] = (pp|qq) - (pq|qp), J[p*N+q] = (pp|qq)
// (global or LDS copies; the additions are the same either way).
__device__ __forceinline__ double h_diag_tab(const double* hd, const double* X, const double* J, int N,
                                             uint64_t a, uint64_t b) {
    double acc = 0.0;
    for (uint64_t x = a; x; x &= x - 1) acc = acc + hd[ctz64(x)];
    for (uint64_t x = b; x; x &= x - 1) acc = acc + hd[ctz64(x)];
    for (uint64_t x = a; x; x &= x - 1) {
        const int p = ctz64(x);
        const double* xr = X + p * N;
        const double* jr = J + p * N;
        for (uint64_t y = x & (x - 1); y; y &= y - 1) acc = acc + xr[ctz64(y)];
        for (uint64_t y = b; y; y &= y - 1) acc = acc + jr[ctz64(y)];
    }
    for (uint64_t x = b; x; x &= x - 1) {
        const double* xr = X + ctz64(x) * N;
        for (uint64_t y = x & (x - 1); y; y &= y - 1) acc = acc + xr[ctz64(y)];
    }
    return acc;
}

__device__ __forceinline__ double h_diag(const SysView& s, uint64_t a, uint64_t b) {
    if (s.onsite) {
        // only opposite-spin pairs on one site contribute; they occur in
        // ascending site order in the canonical pair loop
        double acc = 0.0;
        for (uint64_t x = a; x; x &= x - 1) acc = acc + s.Hd[ctz64(x)];
        for (uint64_t x = b; x; x &= x - 1) acc = acc + s.Hd[ctz64(x)];
        for (uint64_t x = a & b; x; x &= x - 1) acc = acc + s.U[ctz64(x)];
        return acc;
    }
    return h_diag_tab(s.Hd, s.X, s.J, s.N, a, b);
}

// <D2|H|D1> for D1 != D2 by excitation level (zero beyond doubles).
__device__ __forceinline__ double h_offdiag(const SysView& s, uint64_t a1, uint64_t b1, uint64_t a2,
                                            uint64_t b2) {
    const uint64_t ra = a1 & ~a2, rb = b1 & ~b2, xa = a2 & ~a1, xb = b2 & ~b1;
    const int nra = popc64(ra), nrb = popc64(rb);
    if (nra + nrb == 1) {
        if (nra == 1) return h_single(s, a1, b1, 0, ctz64(ra), ctz64(xa));
        return h_single(s, a1, b1, 1, ctz64(rb), ctz64(xb));
    }
    if (nra + nrb != 2) return 0.0;
    int si, pi, sj, pj, sa, pa, sb, pb;
    if (nra == 2) { si = 0; pi = ctz64(ra); sj = 0; pj = ctz64(ra & (ra - 1)); }
    else if (nra == 1) { si = 0; pi = ctz64(ra); sj = 1; pj = ctz64(rb); }
    else { si = 1; pi = ctz64(rb); sj = 1; pj = ctz64(rb & (rb - 1)); }
    const int nxa = popc64(xa);
    if (nxa == 2) { sa = 0; pa = ctz64(xa); sb = 0; pb = ctz64(xa & (xa - 1)); }
    else if (nxa == 1) { sa = 0; pa = ctz64(xa); sb = 1; pb = ctz64(xb); }
    else { sa = 1; pa = ctz64(xb); sb = 1; pb = ctz64(xb & (xb - 1)); }
    return h_double(s, a1, b1, si, pi, sj, pj, sa, pa, sb, pb);
}

// --------------------------------------------------------------------------
// Excitation generators.  Return false for a null draw; otherwise the target
// masks, the generation probability and H_ji.
// --------------------------------------------------------------------------
struct Exc { uint64_t ta, tb; double pgen, H; };

// Uniform singles/doubles with spin imposed by conditional probabilities
// (Appendix A.1).  Random lanes: 0 single/double, 1 electron(s), 2 hole(s).
__device__ __forceinline__ bool gen_uniform(const SysView& s, uint64_t a, uint64_t b, const R4& r,
                                            double p_single, double p_double, Exc& out) {
    const int N = s.N, na = s.na, nb = s.nb, n = s.n;
    const uint64_t full = (N >= 64) ? ~0ULL : low_mask(N);
    if (unif(r.x[0]) < p_single) {
        const int e = (int)pick(r.x[1], (uint64_t)n);
        const int sg = e < na ? 0 : 1;
        const uint64_t occ = sg ? b : a;
        const int pi = select64(occ, sg ? e - na : e);
        const int h = N - (sg ? nb : na);
        if (h == 0) return false;
        const int pa = select64(~occ & full, (int)pick(r.x[2], (uint64_t)h));
        out.pgen = p_single / (double)((uint64_t)n * (uint64_t)h);
        out.H = h_single(s, a, b, sg, pi, pa);
        uint64_t A = a, B = b;
        clear_so(A, B, sg, pi); set_so(A, B, sg, pa);
        out.ta = A; out.tb = B;
        return true;
    }
    if (n < 2) return false;
    const uint64_t npair = (uint64_t)n * (uint64_t)(n - 1) / 2;
    int e1, e2;
    pair_decode(pick(r.x[1], npair), n, e1, e2);
    const int s1 = e1 < na ? 0 : 1, s2 = e2 < na ? 0 : 1;
    const int p1 = select64(s1 ? b : a, s1 ? e1 - na : e1);
    const int p2 = select64(s2 ? b : a, s2 ? e2 - na : e2);
    int sa, pa, sb, pb;
    uint64_t nh;
    if (s1 == s2) {
        const uint64_t holes = ~(s1 ? b : a) & full;
        const int h = N - (s1 ? nb : na);
        if (h < 2) return false;
        nh = (uint64_t)h * (uint64_t)(h - 1) / 2;
        int f1, f2;
        pair_decode(pick(r.x[2], nh), h, f1, f2);
        sa = s1; pa = select64(holes, f1); sb = s1; pb = select64(holes, f2);
    } else {
        const int ha = N - na, hb = N - nb;
        nh = (uint64_t)ha * (uint64_t)hb;
        if (nh == 0) return false;
        const uint64_t q = pick(r.x[2], nh);
        sa = 0; pa = select64(~a & full, (int)(q / (uint64_t)hb));
        sb = 1; pb = select64(~b & full, (int)(q % (uint64_t)hb));
    }
    out.pgen = p_double / (double)(npair * nh);
    out.H = h_double(s, a, b, s1, p1, s2, p2, sa, pa, sb, pb);
    uint64_t A = a, B = b;
    clear_so(A, B, s1, p1); clear_so(A, B, s2, p2); set_so(A, B, sa, pa); set_so(A, B, sb, pb);
    out.ta = A; out.tb = B;
    return true;
}

// Real-space lattice hopping: one of the n electrons, one of the z_p
// neighbours of its site (same spin); null if occupied.  The electron comes
// from the high, the neighbour from the low 32-bit half of word 0 (the
// attempt draws one block; its acceptance is word 1); p_gen is the product
// of the two choices' exact probabilities, 1/(n z_p) for power-of-two counts.
__device__ __forceinline__ bool gen_lattice(const SysView& s, uint64_t a, uint64_t b, const R4& r,
                                            Exc& out) {
    const int N = s.N, na = s.na, n = s.n;
    const int e = (int)pick32((uint32_t)(r.x[0] >> 32), (uint32_t)n);
    const int sg = e < na ? 0 : 1;
    const uint64_t occ = sg ? b : a;
    const int pi = select64(occ, sg ? e - na : e);
    const int z = s.deg[pi];
    if (z == 0) return false;
    const int d = (int)pick32((uint32_t)r.x[0], (uint32_t)z);
    const int q = s.nbr[pi * N + d];
    if ((occ >> q) & 1ULL) return false;
    out.pgen = s.lat_pe[e] * s.lat_pz[z * N + d];
    out.H = h_single(s, a, b, sg, pi, q);
    uint64_t A = a, B = b;
    clear_so(A, B, sg, pi); set_so(A, B, sg, q);
    out.ta = A; out.tb = B;
    return true;
}

// Pre-computed heat-bath doubles (Appendix A.3, Eq. (hbs)) with Walker alias
// tables; uniform singles.  Words of r: 0 single/double and, beyond
// p_single, the pair class (the first p_double p_opp of it: opposite
// spins); 1 electrons; 2 alias column and, from the fraction its pick
// leaves (the low 64 bits of x K, a uniform on a grid of step K / 2^64 for
// every column), the alias coin; 3 acceptance.
// The two pair classes run one code path with per-lane choices (electron
// pair, row, table, column decoding and spins), so that a wave whose lanes
// draw both classes executes it once; each class's arithmetic is the one it
// has on its own.
// p2o, p2s: the class factors p_double p_opp / (n_alpha n_beta) and
// p_double (1 - p_opp) / n_equal-spin-pairs, formed once per step.
__device__ __forceinline__ bool gen_pchb(const SysView& s, uint64_t a, uint64_t b, const R4& r,
                                         double p_single, double p_double, double p_opp, double p2o, double p2s,
                                         Exc& out) {
    const int N = s.N, na = s.na, nb = s.nb;
    const double u0 = unif(r.x[0]);
    if (u0 < p_single) return gen_uniform(s, a, b, r, p_single, p_double, out);
    const uint64_t n_opp = (uint64_t)na * (uint64_t)nb;
    const uint64_t npa = (uint64_t)na * (uint64_t)(na > 0 ? na - 1 : 0) / 2;
    const uint64_t npb = (uint64_t)nb * (uint64_t)(nb > 0 ? nb - 1 : 0) / 2;
    const uint64_t n_same = npa + npb;
    const double pdo = p_double * p_opp;
    const double thr = p_single + pdo;
    const bool opp = u0 < thr;
    const uint64_t ncls = opp ? n_opp : n_same;
    if (ncls == 0) return false;
    const uint64_t q0 = pick(r.x[1], ncls);  // < 2^32
    // electron pair: opposite spins (alpha index q / n_beta, beta q % n_beta);
    // equal spins (pair q of the alpha pairs, then of the beta pairs)
    const int sg = (!opp && q0 >= npa) ? 1 : 0;
    const uint32_t q = (uint32_t)(sg ? q0 - npa : q0);
    int e1, e2;
    if (opp) {
        e1 = (int)div_small(q, s.mnb);
        e2 = (int)(q - (uint32_t)e1 * (uint32_t)nb);
    } else {
        pair_decode(q, sg ? nb : na, e1, e2);
    }
    const uint64_t occ = sg ? b : a;
    const int sI = opp ? 0 : sg, sJ = opp ? 1 : sg;
    const int I = select64(opp ? a : occ, e1);
    const int J = select64(opp ? b : occ, e2);
    const int row = opp ? I * N + J : I * (2 * N - I - 1) / 2 + (J - I - 1);
    const int K = opp ? N * N : N * (N - 1) / 2;
    const uint64_t* tab = opp ? s.hb_opp : s.hb_same;
    const int c0 = (int)pick(r.x[2], (uint64_t)K);
    const uint64_t fx = r.x[2] * (uint64_t)K;  // coin unif(fx): f = fx >> 11
    const size_t at = (size_t)row * (size_t)K + (size_t)c0;
    const uint64_t en = tab[at];
    const uint64_t T = en >> kHbAliasBits, f48 = fx >> 16;
    bool keep = f48 < T;
    if (f48 == T) keep = unif(fx) < (opp ? s.hbp_opp : s.hbp_same)[at];
    const int c = keep ? c0 : (int)(en & ((1u << kHbAliasBits) - 1u));
    int A, Bo;
    if (opp) {
        A = (int)div_small((uint32_t)c, s.mN);
        Bo = c - A * N;
    } else {
        const int ab = s.pair_of[c];
        A = ab >> 6;
        Bo = ab & 63;
    }
    const int sA = sI, sB = sJ;
    const uint64_t mA = sA ? b : a, mB = sB ? b : a;
    if (((mA >> A) & 1ULL) || ((mB >> Bo) & 1ULL)) return false;
    // the column's signed two-electron value, the integral its weight was
    // built from: (AI|BJ), less (AJ|BI) for equal spins, zero where the hole
    // pair meets the electron pair.  p(ab|ij) = w_ab / sum_row with
    // w_ab = |v|; a zero weight (or a zero row) is a null draw.
    const bool z = A == I || Bo == J || (!opp && (A == J || Bo == I));
    const double d = eri(s, A, I, Bo, J);
    const double e = opp ? 0.0 : eri(s, A, J, Bo, I);
    const double v = z ? 0.0 : d - e;
    const double wc = fabs(v);
    if (wc == 0.0) return false;
    const double sum = (opp ? s.hb_sum_opp : s.hb_sum_same)[row];
    const double p2 = opp ? p2o : p2s;
    const double pab = wc / sum;
    out.pgen = p2 * pab;
    out.H = move_pair_parity(a, b, sI, I, sJ, J, A, Bo) ? -v : v;
    uint64_t TA = a, TB = b;
    clear_so(TA, TB, sI, I);
    clear_so(TA, TB, sJ, J);
    set_so(TA, TB, sA, A);
    set_so(TA, TB, sB, Bo);
    out.ta = TA;
    out.tb = TB;
    return true;
}

// On-the-fly Cauchy-Schwarz (EXACT = false) and Part-Exact (EXACT = true)
// generators (Appendix A.2).  Each draw builds its cumulative probability
// functions (CPFs) from N x N tables and the packed integrals:
//  * singles: electron uniform, hole of its spin with weight |H|;
//  * electron pair: first uniform, second from the CPF of |(ii|kk)| times
//    p_opp (opposite spins) or 1 - p_opp; p(ij) = (w_ij/S_i + w_ji/S_j)/n;
//  * opposite spins: beta hole A with weight sqrt((xA|xA)) of the beta
//    electron x, then alpha hole B with sqrt(|(xA|yB)|) (PE) or sqrt((yB|yB))
//    (CS), y the alpha electron;
//  * equal spins x < y: hole A with sqrt((xA|xA)) + sqrt((yA|yA)), then hole
//    B != A with sqrt(|(xA|yB) - (xB|yA)|) (PE) or the first weight (CS);
//    p_gen sums the two hole orders.
// A CPF is inverted at xi = u F_last: the first candidate with F > xi, or the
// last positive weight when rounding leaves none; a zero total is a null
// draw.  Candidates run in canonical order (alpha, then beta; ascending), and
// both passes over a CPF repeat the same additions, so the result is the same
// sequence of binary64 operations as a serial sum.
// Random lanes: r 0 single/double, 1 first electron, 2 second electron (the
// hole for singles), 3 acceptance; r2 0 first hole, 1 second hole.

// Candidate sets m0 (alpha) and m1 (beta); wt(spin, orbital) >= 0.
template <class Wt> __device__ __forceinline__ double cpf_total(uint64_t m0, uint64_t m1, Wt wt) {
    double sum = 0.0;
    for (uint64_t x = m0; x; x &= x - 1) sum = sum + wt(0, ctz64(x));
    for (uint64_t x = m1; x; x &= x - 1) sum = sum + wt(1, ctz64(x));
    return sum;
}

// Returns spin << 6 | orbital of the chosen candidate (-1 if the total is
// zero), its weight in wsel and the total in total.
template <class Wt>
__device__ __forceinline__ int cpf_pick(uint64_t m0, uint64_t m1, Wt wt, double u, double& total,
                                        double& wsel) {
    const double sum = cpf_total(m0, m1, wt);
    total = sum;
    if (sum == 0.0) return -1;
    const double xi = u * sum;
    double acc = 0.0, wl = 0.0;
    int last = -1;
    for (int sp = 0; sp < 2; ++sp) {
        for (uint64_t x = sp ? m1 : m0; x; x &= x - 1) {
            const int p = ctz64(x);
            const double w = wt(sp, p);
            acc = acc + w;
            if (w > 0.0) { last = (sp << 6) | p; wl = w; }
            if (acc > xi) { wsel = w; return (sp << 6) | p; }
        }
    }
    wsel = wl;
    return last;
}

// J and SK are the system's tables of that name, or a copy of them (in LDS).
template <bool EXACT>
__device__ __forceinline__ bool gen_cs(const SysView& s, const double* __restrict__ J,
                                       const double* __restrict__ SK, uint64_t a, uint64_t b, const R4& r,
                                       const R2& r2, double p_single, double p_double, double p_opp, Exc& out) {
    const int N = s.N, na = s.na, n = s.n;
    const uint64_t full = (N >= 64) ? ~0ULL : low_mask(N);
    if (unif(r.x[0]) < p_single) {
        const int e = (int)pick(r.x[1], (uint64_t)n);
        const int sg = e < na ? 0 : 1;
        const uint64_t occ = sg ? b : a;
        const int pi = select64(occ, sg ? e - na : e);
        double tot, wsel;
        const int c = cpf_pick(~occ & full, 0ULL,
                               [&](int, int h) { return fabs(h_single(s, a, b, sg, pi, h)); },
                               unif(r.x[2]), tot, wsel);
        if (c < 0) return false;
        const int pa = c & 63;
        const double p1 = p_single / (double)n;
        out.pgen = p1 * (wsel / tot);
        out.H = h_single(s, a, b, sg, pi, pa);
        uint64_t A = a, B = b;
        clear_so(A, B, sg, pi); set_so(A, B, sg, pa);
        out.ta = A; out.tb = B;
        return true;
    }
    if (n < 2) return false;
    const double q_same = 1.0 - p_opp;
    // electron pair
    const int e1 = (int)pick(r.x[1], (uint64_t)n);
    const int s1 = e1 < na ? 0 : 1;
    const int p1 = select64(s1 ? b : a, s1 ? e1 - na : e1);
    double S1, w12;
    const int c2 = cpf_pick(s1 ? a : a & ~(1ULL << p1), s1 ? b & ~(1ULL << p1) : b,
                            [&](int sk, int pk) { return fabs(J[p1 * N + pk]) * (sk != s1 ? p_opp : q_same); },
                            unif(r.x[2]), S1, w12);
    if (c2 < 0) return false;
    const int s2 = c2 >> 6, p2 = c2 & 63;
    const double S2 = cpf_total(s2 ? a : a & ~(1ULL << p2), s2 ? b & ~(1ULL << p2) : b,
                                [&](int sk, int pk) { return fabs(J[p2 * N + pk]) * (sk != s2 ? p_opp : q_same); });
    const double w21 = fabs(J[p2 * N + p1]) * (s1 != s2 ? p_opp : q_same);
    const double pij = (w12 / S1 + w21 / S2) / (double)n;
    const double pp = p_double * pij;
    // Opposite spins: x the beta electron, y the alpha one, first hole beta;
    // equal spins: x < y, both holes of their spin.  One code path for both,
    // so that the lanes of a wave run the hole loops together.
    const bool opp = s1 != s2;
    const int x = opp ? (s1 ? p1 : p2) : (p1 < p2 ? p1 : p2);
    const int y = opp ? (s1 ? p2 : p1) : (p1 < p2 ? p2 : p1);
    const uint64_t holes_a = ~((opp || s1) ? b : a) & full;
    auto w_first = [&](int, int h) {
        const double u0 = SK[x * N + h];
        if (opp) return u0;
        const double u1 = SK[y * N + h];
        return u0 + u1;
    };
    // second-hole weight given first hole f
    auto w_second = [&](int f, int h) {
        if constexpr (EXACT) {
            const double d = eri(s, x, f, y, h);
            if (opp) return sqrt(fabs(d));
            const double e = eri(s, x, h, y, f);
            return sqrt(fabs(d - e));
        } else {
            if (opp) return SK[y * N + h];
            const double u0 = SK[x * N + h];
            const double u1 = SK[y * N + h];
            return u0 + u1;
        }
    };
    double SA, wA;
    const int cA = cpf_pick(holes_a, 0ULL, w_first, unif(r2.x[0]), SA, wA);
    if (cA < 0) return false;
    const int A = cA & 63;
    const uint64_t holes_b = opp ? ~a & full : holes_a & ~(1ULL << A);
    double SB, wB;
    const int cB = cpf_pick(holes_b, 0ULL, [&](int, int h) { return w_second(A, h); }, unif(r2.x[1]), SB, wB);
    if (cB < 0) return false;
    const int B = cB & 63;
    if (opp) {
        const double q = pp * (wA / SA);
        out.pgen = q * (wB / SB);
        out.H = h_double(s, a, b, 0, y, 1, x, 0, B, 1, A);
        out.ta = (a & ~(1ULL << y)) | (1ULL << B);
        out.tb = (b & ~(1ULL << x)) | (1ULL << A);
        return true;
    }
    // the other order of the holes: B first, then A
    const double SR = cpf_total(holes_a & ~(1ULL << B), 0ULL, [&](int, int h) { return w_second(B, h); });
    const double wAr = w_second(B, A);
    const double wBf = w_first(0, B);
    const double pab = (wA / SA) * (wB / SB);
    const double pba = (wBf / SA) * (wAr / SR);
    out.pgen = pp * (pab + pba);
    const int lo = A < B ? A : B, hi = A < B ? B : A;
    out.H = h_double(s, a, b, s1, x, s1, y, s1, lo, s1, hi);
    const uint64_t occ = s1 ? b : a;
    const uint64_t m = (occ & ~(1ULL << x) & ~(1ULL << y)) | (1ULL << A) | (1ULL << B);
    out.ta = s1 ? a : m;
    out.tb = s1 ? m : b;
    return true;
}

// --------------------------------------------------------------------------
// Wave / block collectives (wave64, 256-thread blocks).
// --------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// Number of set bits of mask in lanes below this one.
__device__ __forceinline__ int lane_rank(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <class T> __device__ __forceinline__ T wave_incl_scan(T v) {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T n = __shfl_up(v, (unsigned)o);
        if (l >= o) v += n;
    }
    return v;
}

template <class T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Exclusive scan over a block of NT threads; `sh` holds NT/64 values.
template <int NT, class T> __device__ __forceinline__ T block_excl_scan(T v, T& total, T* sh) {
    const int w = (int)(threadIdx.x >> 6);
    const T inc = wave_incl_scan(v);
    if (lane_id() == 63) sh[w] = inc;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
        const T x = sh[i];
        if (i < w) off += x;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return off + inc - v;
}

// Four exclusive prefix sums over the workgroup with one exchange (two
// barriers): v[k] becomes the exclusive prefix of v[k], tot[k] the total.
// sh holds 4 * NT/64 values.
template <int NT>
__device__ __forceinline__ void block_excl_scan4(int64_t (&v)[4], int64_t (&tot)[4], int64_t* sh) {
    constexpr int NW = NT / 64;
    const int w = (int)(threadIdx.x >> 6);
    int64_t inc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) inc[k] = wave_incl_scan(v[k]);
    if (lane_id() == 63) {
#pragma unroll
        for (int k = 0; k < 4; ++k) sh[k * NW + w] = inc[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int64_t off = 0, t = 0;
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            const int64_t x = sh[k * NW + i];
            if (i < w) off += x;
            t += x;
        }
        tot[k] = t;
        v[k] = off + inc[k] - v[k];
    }
    __syncthreads();
}

}  // namespace fq
