// Kernels of one FCIQMC step (Eq. fciqmc_dyn: spawn, death, annihilation
// with the initiator rule) on a hash-partitioned walker store.
//
// Walker store: B buckets; determinant D lives in bucket
// floor(hash(D) * B / 2^64).  Bucket b owns R consecutive entries (keys,
// values, cached H_ii - H_00, and the exclusive prefix of the attempt counts)
// plus a count.  Each step reads one store and writes the other.
//
// Per step:
//   k_spawn      one lane per spawn attempt; each record goes straight into
//                the slab of its target bucket (slab sizes reserved from the
//                previous step's counts plus headroom; an overflow replays
//                the step with exact sizes)
//   k_annihilate one workgroup per bucket: death of the bucket's walkers,
//                LDS hash merge of its spawn records under the initiator
//                rule, stochastic rounding, compaction into the other store,
//                estimator partial sums
//   k_post       attempt offsets and record slabs for the next step, global
//                sums, reset of the per-step counters
#pragma once
#include "device.hpp"

namespace fq {

constexpr int kThreads = 256;
constexpr int kChunk = kThreads;     // spawn attempts per workgroup
constexpr int kPostThreads = 512;   // the post kernel's single workgroup
// Each bucket's record slab is split into kSub sub-slabs, each with its own
// counter; workgroup g appends to sub-slab g mod kSub, which divides the
// contention on any one counter by kSub.
constexpr int kSub = 8;
#ifndef FQ_SLOTS
#define FQ_SLOTS 1024
#endif
constexpr int kSlots = FQ_SLOTS;    // LDS hash slots per bucket (table size adapts below this)
constexpr int kSlotsPerThread = kSlots / kThreads;
constexpr int kFresh = 512;         // new determinants per bucket whose diagonal is spread over the workgroup
constexpr int kMaxR = 1024;         // entries per bucket of the walker store

// Spawn chunks of a bucket: its attempts in runs of kChunk (chunks never
// cross buckets, so a chunk's attempts index one bucket's entries).
__host__ __device__ inline int64_t chunks_of(int64_t attempts) { return (attempts + kChunk - 1) / kChunk; }

template <int W, class V> struct Rec {
    uint64_t k[W];
    V v;
    uint32_t flag;  // bit 0: parent is an initiator; bits 1..31: low bits of the key's hash
};

template <class V> struct Store {
    uint64_t* keys;   // B*R*W
    V* vals;          // B*R
    double* diag;     // B*R
    int32_t* mpre;    // B*R: exclusive prefix of attempts within the bucket
    int32_t* count;   // B
    int64_t* batt;    // B: attempts of the bucket
    int64_t* aoff;    // B+1: exclusive prefix of the spawn chunks of the buckets, ceil(batt / kChunk)
};

struct Ctl {
    // accumulated during a step, reset by k_post (or by the host after a failed step)
    unsigned long long nrec;   // spawn records emitted this step
    unsigned int flags;        // kFlag*
    unsigned int pad0;
    double nref;               // C_ref after the step
    // written by k_post
    double nw;
    double enum_;
    long long ndets;
    long long attempts;        // attempts of the next step
    long long nrec_out;
    long long max_count;       // fullest bucket
    double nref_out;
    long long rec_need;        // record slab capacity the next step reserves
    long long chunks;          // spawn chunks (workgroups) of the next step
};

// Record sub-slab for the next step: this step's count plus headroom for
// drift (c/8), for Poisson fluctuations of the count (4 sqrt(c)) and for a
// lump of records that moves between sub-slabs (96): a heavily populated
// parent whose attempts concentrate on a few targets (the heat-bath
// generator does this) puts tens of records into one sub-slab of a bucket,
// and which one follows its chunk index, which shifts from step to step.
// An overflow costs a replay of the whole step.
__device__ __forceinline__ int64_t slab_size(int32_t c) {
    return (int64_t)c + (c >> 3) + (int64_t)(4.0 * sqrt((double)c)) + 96;
}

template <class V> __device__ __forceinline__ double vabs(V v) { return v < 0 ? -(double)v : (double)v; }

// Store of data nobody reads again in this launch (spawn records): marked
// non-temporal, so the scattered lines stream out instead of displacing the
// cached heat-bath tables and parent data.
template <class T> __device__ __forceinline__ void store_stream(T* dst, const T& v) {
    static_assert(sizeof(T) % 8 == 0, "8-byte words");
    uint64_t w[sizeof(T) / 8];
    __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 8); ++i)
        __builtin_nontemporal_store(w[i], reinterpret_cast<uint64_t*>(dst) + i);
}

// a / C_min, the keep probability of the C_min rounding; at the usual
// C_min = 1 the quotient is a itself (exact), and the wave-uniform branch
// skips the division.  The empty asm keeps the compiler from computing the
// quotient ahead of the branch and selecting afterwards.
__device__ __forceinline__ double over_cmin(double a, double c_min) {
    if (c_min == 1.0) return a;
    asm volatile("" : "+v"(a));
    return a / c_min;
}

// Attempts a determinant makes: |C| walkers (integer) or ceil(|C|) (real).
template <class V> __device__ __forceinline__ int64_t n_attempts(V v) {
    if constexpr (sizeof(V) == 4) return v < 0 ? -(int64_t)v : (int64_t)v;
    else return (int64_t)ceil(fabs((double)v));
}

struct StepScalars {
    int64_t t;
    uint64_t seed, replica;
    double tau, p_single, p_double, p_opp, n_a, c_min, S, h00;
    double p2_opp, p2_same;  // heat-bath class factors: p_double p_opp / (n_a n_b), p_double (1 - p_opp) / n_pairs
    uint64_t ref_a, ref_b;
    int B, R;
    long long spawn_cap;
    int import_mode;
    // semi-stochastic deterministic space (ncore = 0: none)
    int64_t ncore;
    const double* core_d;        // (P^D C)_k of this step
    double* core_c;              // C_k after this step, written by the merge
    const uint64_t* core_hkeys;  // open-addressing table of the space: keys (W words a slot)
    const int32_t* core_hidx;    // and indices in the space, -1 for an empty slot
    uint64_t core_hmask;
    // discarded spawns (replica-pair PT2; rej = nullptr: not collected):
    // records of bucket b go to rej[rej_off[b] ...], rej_cnt[b] of them
    void* rej;
    int64_t* rej_off;
    int32_t* rej_cnt;
    // adaptive shift (ada_all = nullptr: off): per record the non-initiator
    // parent's store index (-1 otherwise) and |H|; per input entry the fixed-
    // point sums of accepted and of all spawn weights
    int64_t* rec_par;
    double* rec_h;
    int64_t* ada_acc;
    int64_t* ada_all;
    // replica 2-RDM sampling (rdm_rec = nullptr: off): one record per
    // attempt slot, position chunk * kChunk + lane (RdmRec<W> below)
    void* rdm_rec;
    int64_t rdm_cap;
};

// A generated excitation for the replica 2-RDM: parent (bra) and child
// (ket) determinants and the weight C_i / (m_i p_gen); w = 0 marks an
// attempt slot without a non-null draw.
template <int W> struct RdmRec {
    uint64_t par[W];
    uint64_t chi[W];
    double w;
};

// Fixed point of the adaptive-shift weights: 2^-40 resolution, so integer
// sums of them do not depend on their order.
constexpr double kAdaScale = 1099511627776.0;

// ---------------------------------------------------------------------------
// Semi-stochastic projection (Sec. "Semi-stochastic FCIQMC").  A determinant
// of the deterministic space keeps, in its cached-diagonal slot of the
// walker store, the bits kCoreTag | k: a NaN that no finite diagonal takes,
// carrying its index k in the space.  Entries are copied verbatim, so the
// tag follows the determinant through every step.
// ---------------------------------------------------------------------------
constexpr uint64_t kCoreTag = 0x7FFC000000000000ULL;
__device__ __forceinline__ bool is_core(double d) {
    return ((uint64_t)__double_as_longlong(d) >> 48) == (kCoreTag >> 48);
}
__device__ __forceinline__ int64_t core_index(double d) {
    return (int64_t)((uint64_t)__double_as_longlong(d) & 0xFFFFFFFFFFFFULL);
}
__device__ __forceinline__ double core_tag(int64_t k) { return __longlong_as_double((long long)(kCoreTag | (uint64_t)k)); }

// Index of `key` in the deterministic space, -1 if it is not there (the
// table is at most half full, so the probe meets an empty slot).
template <int W> __device__ __forceinline__ int64_t core_find(const StepScalars& sc, const Key<W>& key) {
    uint64_t s = key_hash<W>(key) & sc.core_hmask;
    for (;;) {
        const int32_t x = sc.core_hidx[s];
        if (x < 0) return -1;
        if (key_eq<W>(load_key<W>(sc.core_hkeys + s * W), key)) return x;
        s = (s + 1) & sc.core_hmask;
    }
}

// ---------------------------------------------------------------------------
// Spawn (Sec. I, step (a)): attempt k of determinant D_i draws an excitation
// D_j with probability p_gen, computes H_ji and spawns with p_s = dtau|H|/p_gen
// (Sec. II).  Attempts are numbered globally by the prefix sums of the
// attempt counts; each lane finds its (bucket, entry, k) by binary search.
// ---------------------------------------------------------------------------
template <int W, class V, int GEN, bool EXT>
__device__ __forceinline__ void spawn_chunk(const SysView& sys, const Store<V>& st, const StepScalars& sc,
                                            Rec<W, V>* __restrict__ rec2, uint64_t* __restrict__ scur, Ctl* ctl,
                                            const int64_t* __restrict__ cmap, int64_t g, int32_t* smpre,
                                            const double* __restrict__ tJ, const double* __restrict__ tSK) {
    // Chunk g is local chunk c of bucket b (cmap[g] = b << 32 | c): the
    // bucket's attempts [c*kChunk, (c+1)*kChunk), one per lane.  The
    // bucket's attempt prefixes are read once into LDS; each lane finds its
    // determinant there.  A record takes the next place of sub-slab
    // j = b'*kSub + g mod kSub of its target bucket b': one atomic add on the
    // sub-slab's cursor word (end << 32 | next place) returns both.
    const Key<W> ref = make_key<W>(sc.ref_a, sc.ref_b);
    const int64_t m = cmap[g];
    const int b = (int)(m >> 32);
    const int64_t eb = (int64_t)b * sc.R;
    const int cnt = st.count[b];
    const int64_t natt = st.batt[b];
    for (int i = threadIdx.x; i < cnt; i += kThreads) smpre[i] = st.mpre[eb + i];
    __syncthreads();
    {
        const int64_t local = (m & 0xFFFFFFFFLL) * kChunk + threadIdx.x;
        bool emit = false;
        Rec<W, V> out;
        int64_t out_parent = -1;  // adaptive shift: non-initiator parent's store index
        double out_h = 0.0;
        uint32_t out_bk = 0;      // target bucket
        RdmRec<W> rdm;            // replica 2-RDM: this slot's draw (w = 0: none)
        rdm.w = 0.0;
        if (local < natt) {
            int elo = 0, ehi = cnt;
            while (ehi - elo > 1) {
                const int mid = (elo + ehi) >> 1;
                if ((int64_t)smpre[mid] <= local) elo = mid; else ehi = mid;
            }
            const int64_t e = eb + elo;
            const uint64_t k = (uint64_t)(local - smpre[elo]);
            const Key<W> key = load_key<W>(st.keys + e * W);
            const V C = st.vals[e];
            const double aC = vabs(C);
            // determinants of the deterministic space count as initiators
            bool pcore = false;
            if constexpr (EXT) pcore = sc.ncore > 0 && is_core(st.diag[e]);
            const bool init = pcore || (sc.n_a < 0.0) || (aC > sc.n_a) || key_eq<W>(key, ref);
            const uint64_t da = key_alpha<W>(key), db = key_beta<W>(key);
            // the attempt's random words, word 3 the acceptance; the lattice
            // generator needs one block (its choices share word 0, its
            // acceptance is the block's word 1)
            R4 r;
            if constexpr (GEN == 1) {
                const R2 q = draw2<W>(key, sc.t, k, kSpawn, sc.seed, sc.replica);
                r.x[0] = q.x[0]; r.x[1] = 0; r.x[2] = 0; r.x[3] = q.x[1];
            } else {
                r = draw<W>(key, sc.t, k, kSpawn, sc.seed, sc.replica);
            }
            Exc x;
            bool ok;
            if constexpr (GEN == 0) ok = gen_uniform(sys, da, db, r, sc.p_single, sc.p_double, x);
            else if constexpr (GEN == 1) ok = gen_lattice(sys, da, db, r, x);
            else if constexpr (GEN == 2)
                ok = gen_pchb(sys, da, db, r, sc.p_single, sc.p_double, sc.p_opp, sc.p2_opp, sc.p2_same, x);
            else {
                const R2 r2 = draw2<W>(key, sc.t, k, kSpawn2, sc.seed, sc.replica);
                ok = gen_cs<GEN == 4>(sys, tJ, tSK, da, db, r, r2, sc.p_single, sc.p_double, sc.p_opp, x);
            }
            if constexpr (EXT) {
                // every non-null draw enters the RDM sample, whatever its fate
                if (ok && sc.rdm_rec) {
                    const double d1 = x.pgen * (double)n_attempts(C);
                    rdm.w = (double)C / d1;
                    const Key<W> tk = make_key<W>(x.ta, x.tb);
#pragma unroll
                    for (int w = 0; w < W; ++w) { rdm.par[w] = key.w[w]; rdm.chi[w] = tk.w[w]; }
                }
                // spawns from the deterministic space into it are part of P^D
                if (ok && pcore && core_find<W>(sc, make_key<W>(x.ta, x.tb)) >= 0) ok = false;
            }
            if (ok && x.H != 0.0) {
                const double u = unif(r.x[3]);
                if constexpr (sizeof(V) == 4) {
                    const double num = sc.tau * fabs(x.H);
                    const double ps = num / x.pgen;
                    const double fl = floor(ps);
                    const double fr = ps - fl;
                    const double nn = fl + (u < fr ? 1.0 : 0.0);
                    if (nn != 0.0) {
                        if (nn > 1073741824.0) atomicOr(&ctl->flags, kFlagBloom);
                        const int32_t m = (int32_t)fmin(nn, 1073741824.0);
                        // child sign -sgn(H) sgn(C): the -dtau H_ji C_i term of Eq. (projector)
                        out.v = ((x.H > 0.0) == (C > 0)) ? -m : m;
                        emit = true;
                    }
                } else {
                    const double x1 = sc.tau * x.H;
                    const double x2 = x1 * (double)C;
                    const double d1 = x.pgen * (double)n_attempts(C);
                    double amp = -(x2 / d1);
                    const double aa = fabs(amp);
                    if (aa < sc.c_min) {
                        const double pr = over_cmin(aa, sc.c_min);
                        amp = (u < pr) ? (amp < 0.0 ? -sc.c_min : sc.c_min) : 0.0;
                    }
                    if (amp != 0.0) { out.v = (V)amp; emit = true; }
                }
                if (emit) {
                    if constexpr (EXT) {
                        if (!init) out_parent = e;
                        out_h = fabs(x.H);
                    }
                    const Key<W> tk = make_key<W>(x.ta, x.tb);
#pragma unroll
                    for (int w = 0; w < W; ++w) out.k[w] = tk.w[w];
                    const uint64_t h = key_hash<W>(tk);
                    out_bk = bucket_of(h, (uint32_t)sc.B);
                    out.flag = (init ? 1u : 0u) | ((uint32_t)h << 1);
                }
            }
        }
        if constexpr (EXT) {
            if (sc.rdm_rec) {
                const int64_t pos = g * kChunk + threadIdx.x;
                if (pos < sc.rdm_cap) static_cast<RdmRec<W>*>(sc.rdm_rec)[pos] = rdm;
                else atomicOr(&ctl->flags, kFlagSpawnCap);
            }
        }
        if (emit) {
            const uint32_t j = out_bk * kSub + (uint32_t)(g & (kSub - 1));
            const uint64_t cw = atomicAdd((unsigned long long*)&scur[j], 1ULL);
            const int64_t pos = (int64_t)(uint32_t)cw;
            if (pos < (int64_t)(cw >> 32) && pos < sc.spawn_cap) {
                store_stream(&rec2[pos], out);
                if (EXT && sc.rec_par) {
                    sc.rec_par[pos] = (out_parent < 0) ? -1 : out_parent;
                    sc.rec_h[pos] = out_h;
                }
            } else {
                atomicOr(&ctl->flags, kFlagSpawnCap);
            }
        }
    }
    __syncthreads();  // smpre is reused by the workgroup's next chunk
}

// Largest orbital count whose J and SK tables the spawn kernel copies to
// LDS (2 N^2 doubles, 32.4 KB at N = 45); larger systems read them from
// global memory.
constexpr int kCsLdsMaxN = 45;

// Waves per SIMD the spawn kernel is compiled for: the table-driven
// generators fit eight (its latency-bound gathers want every wave the SIMD
// holds), at the price of a few scalar registers kept in vector lanes; the
// on-the-fly generators keep the compiler's own choice rather than spill.
template <int GEN> constexpr int kSpawnWaves = GEN <= 2 ? 8 : 1;

template <int W, class V, int GEN, bool EXT>
__global__ __launch_bounds__(kThreads, kSpawnWaves<GEN>) void k_spawn(SysView sys, Store<V> st, StepScalars sc,
                                                    Rec<W, V>* __restrict__ rec2,
                                                    uint64_t* __restrict__ scur, Ctl* ctl,
                                                    const int64_t* __restrict__ cmap, int64_t cmap_cap) {
    // the chunk count of this step comes from the post work of the previous
    // one, so a launch may be queued before the host has read it
    __shared__ int32_t smpre[kMaxR];
    const int64_t n = ctl->chunks;
    if (n > cmap_cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&ctl->flags, kFlagSpawnCap);
        return;
    }
    if (GEN >= 3 && sys.N <= kCsLdsMaxN) {
        // the Cauchy-Schwarz generators read J and SK for every candidate
        // electron and hole: both N x N tables are copied to LDS (dynamic
        // shared memory of 2 N^2 doubles) once per workgroup; the loop is
        // its own copy so that its table reads compile to LDS loads
        extern __shared__ double cs_tab[];
        const int nn = sys.N * sys.N;
        for (int i = threadIdx.x; i < nn; i += kThreads) {
            cs_tab[i] = sys.J[i];
            cs_tab[nn + i] = sys.SK[i];
        }
        __syncthreads();
        for (int64_t g = blockIdx.x; g < n; g += gridDim.x)
            spawn_chunk<W, V, GEN, EXT>(sys, st, sc, rec2, scur, ctl, cmap, g, smpre, cs_tab, cs_tab + nn);
        return;
    }
    for (int64_t g = blockIdx.x; g < n; g += gridDim.x)
        spawn_chunk<W, V, GEN, EXT>(sys, st, sc, rec2, scur, ctl, cmap, g, smpre, sys.J, sys.SK);
}

// Records uploaded from the host (population import): assign buckets.
template <int W, class V>
__global__ __launch_bounds__(kThreads) void k_bucketize(Rec<W, V>* rec, long long n, int B,
                                                        int32_t* scount) {
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (long long)gridDim.x * kThreads) {
        Key<W> k;
#pragma unroll
        for (int w = 0; w < W; ++w) k.w[w] = rec[i].k[w];
        const uint64_t h = key_hash<W>(k);
        const uint32_t b = bucket_of(h, (uint32_t)B);
        rec[i].flag = (rec[i].flag & 1u) | ((uint32_t)h << 1);
        atomicAdd(&scount[b * kSub + (uint32_t)(i & (kSub - 1))], 1);
    }
}

// Record slabs from per-bucket counts (one workgroup of 1024 threads, each
// scanning a contiguous segment): soff = exclusive prefix of the counts, or
// of slab_size(count) when `headroom` is set; the counts are then zeroed
// and the cursor words set (end << 32 | start).
__device__ __forceinline__ void offsets_from_counts(int32_t* __restrict__ cnt, int B, int headroom,
                                                    int64_t* __restrict__ off, uint64_t* __restrict__ cur,
                                                    long long* total_out, long long* count_out, int64_t* sh) {
    const int T = 1024;
    const int per = (B + T - 1) / T;
    const int s0 = threadIdx.x * per;
    const int s1 = min(B, s0 + per);
    int64_t loc = 0, raw = 0;
    for (int i = s0; i < s1; ++i) {
        loc += headroom ? slab_size(cnt[i]) : (int64_t)cnt[i];
        raw += cnt[i];
    }
    int64_t tot;
    int64_t run = block_excl_scan<1024, int64_t>(loc, tot, sh);
    int64_t rtot;
    (void)block_excl_scan<1024, int64_t>(raw, rtot, sh);
    for (int i = s0; i < s1; ++i) {
        off[i] = run;
        const int64_t e = run + (headroom ? slab_size(cnt[i]) : (int64_t)cnt[i]);
        cur[i] = ((uint64_t)e << 32) | (uint64_t)run;
        run = e;
        cnt[i] = 0;
    }
    if (threadIdx.x == 0) {
        off[B] = tot;
        *total_out = tot;
        if (count_out) *count_out = rtot;
    }
}

__global__ __launch_bounds__(1024) void k_offsets(int32_t* __restrict__ cnt, int B, int headroom,
                                                  int64_t* __restrict__ off, uint64_t* __restrict__ cur, Ctl* ctl) {
    __shared__ int64_t sh[16];
    offsets_from_counts(cnt, B, headroom, off, cur, &ctl->rec_need, (long long*)nullptr, sh);
}

// Cursors back to their sub-slab starts (the end halves are untouched by a
// spawn), after a queued spawn launch is dropped.
__global__ void k_slab_rewind(uint64_t* __restrict__ cur, const int64_t* __restrict__ off, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        cur[i] = (cur[i] & 0xFFFFFFFF00000000ULL) | (uint64_t)(uint32_t)off[i];
}

// Records each sub-slab received (cursor minus start; a full sub-slab's
// cursor counts on past its end), for slabs rebuilt after an overflow.
__global__ void k_slab_counts(const uint64_t* __restrict__ cur, const int64_t* __restrict__ off, int n,
                              int32_t* __restrict__ cnt) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        cnt[i] = (int32_t)((uint32_t)cur[i] - (uint32_t)off[i]);
}

// Exclusive prefix of counts into offsets without modifying the counts.
__global__ __launch_bounds__(1024) void k_count_offsets(const int32_t* __restrict__ cnt, int B,
                                                        int64_t* __restrict__ off) {
    __shared__ int64_t sh[16];
    const int T = 1024;
    const int per = (B + T - 1) / T;
    const int s0 = threadIdx.x * per;
    const int s1 = min(B, s0 + per);
    int64_t loc = 0;
    for (int i = s0; i < s1; ++i) loc += cnt[i];
    int64_t tot;
    int64_t run = block_excl_scan<1024, int64_t>(loc, tot, sh);
    for (int i = s0; i < s1; ++i) { off[i] = run; run += cnt[i]; }
    if (threadIdx.x == 0) off[B] = tot;
}

// Imported records (flat array, buckets assigned) into their slabs.
template <int W, class V>
__global__ __launch_bounds__(kThreads) void k_scatter(const Rec<W, V>* __restrict__ rec, long long n, int B,
                                                      Rec<W, V>* __restrict__ rec2,
                                                      uint64_t* __restrict__ scur) {
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (long long)gridDim.x * kThreads) {
        const Rec<W, V> r = rec[i];
        Key<W> k;
#pragma unroll
        for (int w = 0; w < W; ++w) k.w[w] = r.k[w];
        const uint32_t j = bucket_of(key_hash<W>(k), (uint32_t)B) * kSub + (uint32_t)(i & (kSub - 1));
        const int64_t pos = (int64_t)(uint32_t)atomicAdd((unsigned long long*)&scur[j], 1ULL);
        rec2[pos] = r;
    }
}

// ---------------------------------------------------------------------------
// LDS hash table of one bucket.
// ---------------------------------------------------------------------------
template <int W, class V> struct LdsTable {
    uint64_t key0[kSlots];
    uint64_t key1[W == 2 ? kSlots : 1];
    V val[kSlots];
    int16_t idx[kSlots];   // entry index in the input store (< R), -1 for a new determinant
};

// New survivors of lattice systems awaiting their diagonal (slot | out
// position << 11); one-word layouts only, two-word lattice stores compute
// theirs inline.
template <int W> constexpr int fresh_cap() { return W == 1 ? kFresh : 0; }

template <int W, class V> struct Lds {
    LdsTable<W, V> t;
    int32_t fresh[W == 1 ? kFresh : 1];
    int nfresh;
    int64_t sh64[8];
    double shd[8];
};

template <int W> __device__ __forceinline__ uint64_t lds_load(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Find the slot of `key` in an LDS table T (arrays key0, and key1 for
// two-word keys); insert it if absent and `insert` is set.  Returns the
// slot, -1 if absent (not inserted), -2 if the table is full, -3 if a
// claimed slot never became readable.
template <int W, class T>
__device__ __forceinline__ int lds_find(T& tab, const Key<W>& key, uint64_t h, uint64_t mask, bool insert) {
    int s = (int)(h & mask);
    int probes = 0;
    int spins = 0;
    while (true) {
        uint64_t w0 = lds_load<W>(&tab.key0[s]);
        if (w0 == kEmpty) {
            if (!insert) return -1;
            if constexpr (W == 1) {
                const uint64_t old = atomicCAS((unsigned long long*)&tab.key0[s], kEmpty, key.w[0]);
                if (old == kEmpty || old == key.w[0]) return s;
                w0 = old;
            } else {
                const uint64_t old = atomicCAS((unsigned long long*)&tab.key0[s], kEmpty, kLocked);
                if (old == kEmpty) {
                    __hip_atomic_store(&tab.key1[s], key.w[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    __hip_atomic_store(&tab.key0[s], key.w[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    return s;
                }
                w0 = old;
            }
        }
        if constexpr (W == 2) {
            if (w0 == kLocked) {
                // retry the same slot in the next pass of this loop, so the
                // claiming lane (possibly in this wave) publishes first
                if (++spins > (1 << 22)) return -3;
                continue;
            }
            if (w0 == key.w[0]) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                if (lds_load<W>(&tab.key1[s]) == key.w[1]) return s;
            }
        } else {
            if (w0 == key.w[0]) return s;
        }
        s = (s + 1) & (int)mask;
        // every slot visited: a full table cannot take the key, and a lookup
        // has seen every key there is (one that runs while other lanes still
        // insert may find the table full only because of them)
        if (++probes > (int)mask) return insert ? -2 : -1;
    }
}

// Insert `key`, known to differ from every key inserted before or alongside
// it, into an LDS table that no lane reads until the next barrier: the
// first empty slot of its probe sequence, taken by one compare-and-swap of
// the first word (the second is a plain store, visible after the barrier).
// Returns the slot, -2 if the table is full.
template <int W, class T>
__device__ __forceinline__ int lds_insert_new(T& tab, const Key<W>& key, uint64_t h, uint64_t mask) {
    int s = (int)(h & mask);
    for (int probes = 0; probes <= (int)mask; ++probes) {
        const uint64_t old = atomicCAS((unsigned long long*)&tab.key0[s], kEmpty, key.w[0]);
        if (old == kEmpty) {
            if constexpr (W == 2) tab.key1[s] = key.w[1];
            return s;
        }
        s = (s + 1) & (int)mask;
    }
    return -2;
}

template <class V> __device__ __forceinline__ void lds_add(V* p, V v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Sub-slab j of bucket b holds records [base + r[j], base + r[j+1]) (r[kSub]
// = need, the bucket's slab size): its start, and its cursor word for the
// spawn (end << 32 | start).
__device__ __forceinline__ void set_subslab(int64_t* __restrict__ soff, uint64_t* __restrict__ scur, int b, int j,
                                            int64_t start, int64_t end) {
    soff[(int64_t)b * kSub + j] = start;
    scur[(int64_t)b * kSub + j] = ((uint64_t)end << 32) | (uint64_t)start;
}

// ---------------------------------------------------------------------------
// Global sums and next-step offsets (attempt prefix over buckets, record
// sub-slab offsets), executed by one workgroup of NT threads, then the step
// scalars written to `host` (pinned host memory).  The flag word, the
// reference amplitude and the per-bucket values are loaded together, and the
// host copy is composed from registers, so the kernel waits on memory twice
// (loads, then the final stores) instead of once per stage.  A flagged step
// writes no offsets; its host copy is the control block as the step left it.
// ---------------------------------------------------------------------------
template <int NT, int HELD = 2>
__device__ __forceinline__ void post_work(const int64_t* __restrict__ batt, const int32_t* __restrict__ count,
                                          const double* __restrict__ nw_b, const double* __restrict__ en_b,
                                          const int64_t* __restrict__ rel, const int64_t* __restrict__ need_b,
                                          const int64_t* __restrict__ recs_b, int B,
                                          int64_t* __restrict__ aoff, int64_t* __restrict__ soff,
                                          uint64_t* __restrict__ scur,
                                          int64_t* __restrict__ cmap, int64_t cmap_cap, Ctl* ctl,
                                          Ctl* __restrict__ host, int64_t* sh, double* shd, int64_t* shm,
                                          unsigned* shf) {
    double nref = 0.0;
    if (threadIdx.x == 0) {
        *shf = __hip_atomic_load(&ctl->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        nref = ctl->nref;
    }
    // one pass of loads (all per-bucket values of this thread's run of
    // buckets), the scans, then one pass of writes
    const int per = (B + NT - 1) / NT;
    const int b0 = threadIdx.x * per, b1 = min(B, b0 + per);
    int64_t la = 0, lk = 0, ln = 0, cnt = 0, rc = 0, mx = 0;
    double nw = 0.0, en = 0.0;
    // the first kHeld buckets of the run keep what the offset pass needs in
    // registers (no second round of loads after the scan); kHeld = 0 keeps
    // none, for kernels whose other work needs the registers
    constexpr int kHeld = HELD;
    int64_t hatt[kHeld > 0 ? kHeld : 1] = {}, hneed[kHeld > 0 ? kHeld : 1] = {},
            hrel[kHeld > 0 ? kHeld : 1][kSub] = {};
    auto add = [&](int b, int64_t at, int64_t nd) {
        la += at;
        lk += chunks_of(at);
        ln += nd;
        const int64_t c = count[b];
        cnt += c;
        rc += recs_b[b];
        mx = max(mx, c);
        nw = nw + nw_b[b];
        en = en + en_b[b];
    };
#pragma unroll
    for (int i = 0; i < kHeld; ++i) {
        const int b = b0 + i;
        if (b < b1) {
            hatt[i] = batt[b];
            hneed[i] = need_b[b];
#pragma unroll
            for (int j = 0; j < kSub; ++j) hrel[i][j] = rel[(int64_t)b * kSub + j];
            add(b, hatt[i], hneed[i]);
        }
    }
    for (int b = b0 + kHeld; b < b1; ++b) add(b, batt[b], need_b[b]);
    // attempts, chunks, slab sizes, and determinants (< 2^32) with records
    // (< 2^31 per step) packed: four prefix sums in one exchange (whose
    // barrier also publishes the flag word)
    int64_t v[4] = {la, lk, ln, (cnt << 32) | rc};
    int64_t tot[4];
    block_excl_scan4<NT>(v, tot, sh);
    const unsigned flags = *shf;
    const int64_t atot = tot[0], ktot = tot[1], ntot = tot[2], crtot = tot[3];
    if (flags == 0) {
        int64_t run = v[1], base = v[2];
#pragma unroll
        for (int i = 0; i < kHeld; ++i) {
            const int b = b0 + i;
            if (b < b1) {
                aoff[b] = run;
                const int64_t nk = chunks_of(hatt[i]);
                for (int64_t c = 0; c < nk && run + c < cmap_cap; ++c) cmap[run + c] = ((int64_t)b << 32) | c;
                run += nk;
#pragma unroll
                for (int j = 0; j < kSub; ++j)
                    set_subslab(soff, scur, b, j, base + hrel[i][j], base + (j + 1 < kSub ? hrel[i][j + 1] : hneed[i]));
                base += hneed[i];
            }
        }
        for (int b = b0 + kHeld; b < b1; ++b) {
            aoff[b] = run;
            const int64_t nk = chunks_of(batt[b]);
            for (int64_t c = 0; c < nk && run + c < cmap_cap; ++c) cmap[run + c] = ((int64_t)b << 32) | c;
            run += nk;
            int64_t r0 = rel[(int64_t)b * kSub];
            for (int j = 0; j < kSub; ++j) {
                const int64_t r1 = j + 1 < kSub ? rel[(int64_t)b * kSub + j + 1] : need_b[b];
                set_subslab(soff, scur, b, j, base + r0, base + r1);
                r0 = r1;
            }
            base += need_b[b];
        }
    }
    // N_w and the E_proj numerator in a fixed order: per-thread runs, wave
    // butterflies, waves in order
    nw = wave_sum(nw);
    en = wave_sum(en);
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, (int64_t)__shfl_xor(mx, o));
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) { shd[w] = nw; shd[NT / 64 + w] = en; shm[w] = mx; }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (flags != 0) {
            *host = *ctl;
        } else {
            double a = 0.0, c = 0.0;
            int64_t m = 0;
            for (int i = 0; i < NT / 64; ++i) { a = a + shd[i]; c = c + shd[NT / 64 + i]; m = max(m, shm[i]); }
            aoff[B] = ktot;
            soff[(int64_t)B * kSub] = ntot;
            Ctl h;
            h.nrec = 0;
            h.flags = 0;
            h.pad0 = 0;
            h.nref = 0.0;
            h.nw = a;
            h.enum_ = c;
            h.ndets = crtot >> 32;
            h.attempts = atot;
            h.nrec_out = crtot & 0xFFFFFFFFLL;
            h.max_count = m;
            h.nref_out = nref;
            h.rec_need = ntot;
            h.chunks = ktot;
            *ctl = h;
            *host = h;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Death, annihilation with the initiator rule, compaction and estimators,
// one workgroup per bucket (Sec. I steps (b) and (c); Sec. IV Eq. (proje)).
// ---------------------------------------------------------------------------
constexpr int64_t kM40 = (1LL << 40) - 1;

// Place in the record buffer of a bucket's q-th record, its sub-slabs
// walked as one sequence: cum[j] records precede sub-slab j (ascending), and
// base[j] is the sub-slab's start less cum[j].  Each sub-slab's range is
// tested on its own (unrolled selects of register values; a select of the
// last sub-slab with cum[j] <= q compiles to an indexed private-memory load).
__device__ __forceinline__ int64_t rec_place(const int64_t* base, const int32_t* cum, int32_t q) {
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < kSub; ++j)
        if (q >= cum[j] && q < cum[j + 1]) s = base[j];
    return s + q;
}

// The step's flag word, read once for the whole workgroup so that every wave
// takes the same branch (another workgroup may set a flag meanwhile).
__device__ __forceinline__ unsigned wg_flags(const Ctl* ctl, unsigned* sh) {
    if (threadIdx.x == 0) *sh = __hip_atomic_load(&ctl->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const unsigned f = *sh;
    __syncthreads();
    return f;
}

template <int W, class V, bool EXT>
__device__ __forceinline__ void annihilate_bucket(const SysView& sys, const Store<V>& in, const Store<V>& out,
                                                  const StepScalars& sc, const Rec<W, V>* __restrict__ rec2,
                                                  const int64_t* __restrict__ soff, const uint64_t* __restrict__ scur,
                                                  int64_t* __restrict__ rel, int64_t* __restrict__ need_b,
                                                  int64_t* __restrict__ recs_b, double* __restrict__ nw_b,
                                                  double* __restrict__ en_b, uint16_t* __restrict__ fpos,
                                                  int32_t* __restrict__ fcnt, Ctl* ctl, int b, Lds<W, V>& L) {
    const Key<W> ref = make_key<W>(sc.ref_a, sc.ref_b);
    constexpr bool kInt = sizeof(V) == 4;
    const int64_t eb = (int64_t)b * sc.R;
    const int cnt = sc.import_mode ? 0 : in.count[b];
    // the bucket's records: its kSub sub-slabs, walked as one sequence
    // (cumulative counts and starts held in registers)
    int64_t lo[kSub], base[kSub];
    int32_t cj[kSub], cum[kSub + 1];
    cum[0] = 0;
#pragma unroll
    for (int j = 0; j < kSub; ++j) {
        lo[j] = soff[(int64_t)b * kSub + j];
        cj[j] = (int32_t)((uint32_t)scur[(int64_t)b * kSub + j] - (uint32_t)lo[j]);
        cum[j + 1] = cum[j] + cj[j];
        base[j] = lo[j] - cum[j];
    }
    const int32_t nrec = cum[kSub];
    // LDS table sized to the bucket: keys <= determinants + records, load <= 3/4
    const int64_t want = ((int64_t)cnt + nrec) * 4 / 3 + 1;
    int nslots = kThreads;
    while (nslots < want && nslots < kSlots) nslots <<= 1;
    const uint64_t mask = (uint64_t)(nslots - 1);
    // this thread's first determinant and first two records are loaded now,
    // so their latency overlaps the table reset and the death pass
    const int e0 = (int)threadIdx.x;
    Key<W> pk;
    V pC = (V)0;
    double pd = 0.0;
    if (e0 < cnt) {
        pk = load_key<W>(in.keys + (eb + e0) * W);
        pC = in.vals[eb + e0];
        pd = in.diag[eb + e0];
    }
    Rec<W, V> prec, prec2;
    if (e0 < nrec) prec = rec2[rec_place(base, cum, e0)];
    if (e0 + kThreads < nrec) prec2 = rec2[rec_place(base, cum, e0 + kThreads)];
    for (int i = threadIdx.x; i < nslots; i += kThreads) {
        L.t.key0[i] = kEmpty;
        if constexpr (W == 2) L.t.key1[i] = kEmpty;
        L.t.val[i] = (V)0;
        L.t.idx[i] = -1;
    }
    if (threadIdx.x == 0) L.nfresh = 0;
    __syncthreads();
    // (b) death of the walkers occupied at tau: x = (1 - dtau (d_i - S)) C_i,
    // stochastically rounded; the slot is marked as occupied at tau.  The
    // first determinant is the prefetched one.
    auto death = [&](const Key<W>& key, const V C, const double d, const int e) {
        V post;
        if (EXT && sc.ncore > 0 && is_core(d)) {
            // deterministic space: P^D C, diagonal included, unrounded
            post = (V)sc.core_d[core_index(d)];
        } else {
            double Sx = sc.S;
            if (EXT && sc.ada_all) {
                // adaptive shift: a non-initiator's local shift f S
                const bool ini = (sc.n_a < 0.0) || (vabs(C) > sc.n_a) || key_eq<W>(key, ref);
                const int64_t T = sc.ada_all[eb + e];
                if (!ini && T > 0) {
                    const double f = (double)sc.ada_acc[eb + e] / (double)T;
                    Sx = f * sc.S;
                }
            }
            const double t1 = d - Sx;
            const double t2 = sc.tau * t1;
            const double f = 1.0 - t2;
            const double xv = f * (double)C;
            const double u = unif(draw2<W>(key, sc.t, 0, kDeath, sc.seed, sc.replica).x[0]);
            if constexpr (kInt) {
                const double ax = fabs(xv);
                const double fl = floor(ax);
                const double fr = ax - fl;
                const double nn = fl + (u < fr ? 1.0 : 0.0);
                if (nn > 2147483000.0) atomicOr(&ctl->flags, kFlagPop);
                post = (V)(xv < 0.0 ? -nn : nn);
            } else {
                const double ax = fabs(xv);
                double y = xv;
                if (ax < sc.c_min && xv != 0.0) {
                    const double pr = over_cmin(ax, sc.c_min);
                    y = (u < pr) ? (xv < 0.0 ? -sc.c_min : sc.c_min) : 0.0;
                }
                post = (V)y;
            }
        }
        // the bucket's walkers are distinct determinants
        const int s = lds_insert_new<W>(L.t, key, key_hash<W>(key), mask);
        if (s < 0) { atomicOr(&ctl->flags, kFlagTable); return; }
        L.t.val[s] = post;
        L.t.idx[s] = e;
    };
    if (e0 < cnt) death(pk, pC, pd, e0);
    for (int e = e0 + kThreads; e < cnt; e += kThreads)
        death(load_key<W>(in.keys + (eb + e) * W), in.vals[eb + e], in.diag[eb + e], e);
    __syncthreads();
    // (c) annihilation: a target occupied at tau takes every contribution;
    // an unoccupied one only those of initiator parents (Sec. I).  The first
    // two records are the prefetched ones.
    auto merge = [&](const Rec<W, V>& x) {
        Key<W> key;
#pragma unroll
        for (int w = 0; w < W; ++w) key.w[w] = x.k[w];
        const bool init = (x.flag & 1u) != 0;
        const int s = lds_find<W>(L.t, key, (uint64_t)(x.flag >> 1), mask, init);
        if (s == -1) return;
        if (s < 0) { atomicOr(&ctl->flags, s == -2 ? kFlagTable : kFlagSpin); return; }
        if (init || L.t.idx[s] >= 0) lds_add<V>(&L.t.val[s], x.v);
    };
    if (e0 < nrec) merge(prec);
    if (e0 + kThreads < nrec) merge(prec2);
    for (int32_t q = e0 + 2 * kThreads; q < nrec; q += kThreads) merge(rec2[rec_place(base, cum, q)]);
    __syncthreads();
    if (EXT && sc.rej != nullptr && !sc.import_mode) {
        // discarded spawns: non-initiator records whose target is in neither
        // the population at tau nor the new one (no initiator spawn reached
        // it), kept in record order in the bucket's region of the buffer
        Rec<W, V>* rej = static_cast<Rec<W, V>*>(sc.rej);
        int64_t nb = 0;
        for (int32_t q0 = 0; q0 < nrec; q0 += kThreads) {
            const int32_t q = q0 + (int32_t)threadIdx.x;
            bool dropped = false;
            Rec<W, V> x;
            if (q < nrec) {
                x = rec2[rec_place(base, cum, q)];
                if (!(x.flag & 1u)) {
                    Key<W> key;
#pragma unroll
                    for (int w = 0; w < W; ++w) key.w[w] = x.k[w];
                    dropped = lds_find<W>(L.t, key, (uint64_t)(x.flag >> 1), mask, false) == -1;
                }
            }
            int64_t tot;
            const int64_t ex = block_excl_scan<kThreads, int64_t>(dropped ? 1 : 0, tot, L.sh64);
            if (dropped) rej[lo[0] + nb + ex] = x;
            nb += tot;
        }
        if (threadIdx.x == 0) {
            sc.rej_off[b] = lo[0];
            sc.rej_cnt[b] = (int32_t)nb;
        }
    }
    if (threadIdx.x < kSub) {
        // slabs of the next step: this step's counts plus headroom, relative
        // to the bucket's base (the post work places them and sets the
        // cursors).  Lane j sizes sub-slab j; an 8-lane scan places them.
        const int j = (int)threadIdx.x;
        if (!sc.import_mode) {
            int32_t c = 0;
#pragma unroll
            for (int i = 0; i < kSub; ++i)
                if (i == j) c = cj[i];
            const long long sz = slab_size(c);
            long long inc = sz;
#pragma unroll
            for (int o = 1; o < kSub; o <<= 1) {
                const long long t = __shfl_up(inc, o, kSub);
                if (j >= o) inc += t;
            }
            rel[(int64_t)b * kSub + j] = inc - sz;
            if (j == kSub - 1) need_b[b] = inc;
        }
        if (j == 0) recs_b[b] = nrec;
    }
    // compaction: (1) each thread rounds its run of nslots / kThreads
    // consecutive slots in place (small real amplitudes) and drops what it
    // does not keep; (2) one block scan of (kept << 40 | attempts) over the
    // runs gives each run's output position and attempt prefix, so the
    // output stays in slot order; (3) the runs are written out.
    const int run_len = nslots / kThreads;
    const int s0 = (int)threadIdx.x * run_len;
    int64_t mine = 0;
    for (int j = 0; j < run_len; ++j) {
        const int s = s0 + j;
        const uint64_t k0 = L.t.key0[s];
        if (k0 == kEmpty) continue;
        V v = L.t.val[s];
        bool core = false;
        if (EXT && sc.ncore > 0 && L.t.idx[s] >= 0) core = is_core(in.diag[eb + L.t.idx[s]]);
        if constexpr (!kInt) {
            const double av = fabs((double)v);
            if (!core && !sc.import_mode && v != 0.0 && av < sc.c_min) {
                Key<W> key;
                key.w[0] = k0;
                if constexpr (W == 2) key.w[1] = L.t.key1[s];
                const double u = unif(draw2<W>(key, sc.t, 0, kAnn, sc.seed, sc.replica).x[0]);
                const double pr = over_cmin(av, sc.c_min);
                v = (u < pr) ? (v < 0.0 ? -sc.c_min : sc.c_min) : 0.0;
                L.t.val[s] = v;
            }
        }
        // the deterministic space stays at any value; an import keeps every
        // entry it was given
        const bool keep = v != (V)0 || core || sc.import_mode;
        if (keep) mine += (1LL << 40) | n_attempts(v);
        else L.t.key0[s] = kEmpty;
    }
    int64_t tot;
    const int64_t ex = block_excl_scan<kThreads, int64_t>(mine, tot, L.sh64);
    const int64_t obase = tot >> 40, mbase = tot & kM40;
    const bool over = obase > sc.R || mbase >= (int64_t)0x7FFFFFFF;
    double nw = 0.0, en = 0.0;
    if (!over) {
        int64_t pos = ex >> 40, mp = ex & kM40;
        for (int j = 0; j < run_len; ++j) {
            const int s = s0 + j;
            const uint64_t k0 = L.t.key0[s];
            if (k0 == kEmpty) continue;
            Key<W> key;
            key.w[0] = k0;
            if constexpr (W == 2) key.w[1] = L.t.key1[s];
            const V v = L.t.val[s];
            const int64_t o = eb + pos;
            store_key<W>(out.keys + o * W, key);
            out.vals[o] = v;
            out.mpre[o] = (int32_t)mp;
            const int oi = L.t.idx[s];
            if constexpr (EXT) {
                // adaptive shift: the next step's accumulators start at zero
                // (this bucket's death pass has read the old ones)
                if (sc.ada_all) { sc.ada_acc[o] = 0; sc.ada_all[o] = 0; }
                if (sc.ncore > 0 && oi >= 0) {
                    const double dd = in.diag[eb + oi];
                    if (is_core(dd)) sc.core_c[core_index(dd)] = (double)v;
                }
            }
            const uint64_t ka = key_alpha<W>(key), kb = key_beta<W>(key);
            if (oi >= 0) {
                out.diag[o] = in.diag[eb + oi];
            } else if (sys.onsite) {
                // new determinant of a lattice system: its (short) diagonal is
                // computed below, spread over the workgroup
                const int f = atomicAdd(&L.nfresh, 1);
                if (f < fresh_cap<W>()) L.fresh[f] = s | ((int)pos << 11);
                else { const double hd = h_diag(sys, ka, kb); out.diag[o] = hd - sc.h00; }
            } else {
                // new determinant: listed for the diagonal kernel (k_fresh)
                const int f = atomicAdd(&L.nfresh, 1);
                fpos[eb + f] = (uint16_t)pos;
            }
            const double av = vabs(v);
            nw = nw + av;
            if (key_eq<W>(key, ref)) {
                ctl->nref = (double)v;
            } else {
                const int lvl = popc64(ka ^ sc.ref_a) + popc64(kb ^ sc.ref_b);
                if (lvl == 2 || lvl == 4) {
                    const double h = h_offdiag(sys, sc.ref_a, sc.ref_b, ka, kb);
                    const double c = h * (double)v;
                    en = en + c;
                }
            }
            pos += 1;
            mp += n_attempts(v);
        }
    }
    if (over) {
        if (threadIdx.x == 0) atomicOr(&ctl->flags, kFlagStore);
        __syncthreads();
        return;
    }
    nw = wave_sum(nw);
    en = wave_sum(en);
    if (lane_id() == 0) { L.shd[threadIdx.x >> 6] = nw; L.shd[4 + (threadIdx.x >> 6)] = en; }
    __syncthreads();
    if (sys.onsite) {
        // diagonals of new lattice determinants, spread over the workgroup
        const int nf = min(L.nfresh, fresh_cap<W>());
#pragma unroll
        for (int i = 0; i < fresh_cap<W>() / kThreads; ++i) {
            const int f = threadIdx.x + i * kThreads;
            if (f >= nf) continue;
            const int s = L.fresh[f] & 2047;
            Key<W> fk;
            fk.w[0] = L.t.key0[s];
            if constexpr (W == 2) fk.w[1] = L.t.key1[s];
            const double h = h_diag(sys, key_alpha<W>(fk), key_beta<W>(fk));
            out.diag[eb + (L.fresh[f] >> 11)] = h - sc.h00;
        }
    } else if (threadIdx.x == 0) {
        fcnt[b] = L.nfresh;
    }
    if (threadIdx.x == 0) {
        nw_b[b] = ((L.shd[0] + L.shd[1]) + L.shd[2]) + L.shd[3];
        en_b[b] = ((L.shd[4] + L.shd[5]) + L.shd[6]) + L.shd[7];
        out.count[b] = (int32_t)obase;
        out.batt[b] = mbase;
    }
    __syncthreads();
}

template <int W, class V, bool EXT>
__global__ __launch_bounds__(kThreads, 6) void k_annihilate(SysView sys, Store<V> in, Store<V> out,
                                                         StepScalars sc,
                                                         const Rec<W, V>* __restrict__ rec2,
                                                         const int64_t* __restrict__ soff,
                                                         const uint64_t* __restrict__ scur,
                                                         int64_t* __restrict__ rel,
                                                         int64_t* __restrict__ need_b,
                                                         int64_t* __restrict__ recs_b,
                                                         double* __restrict__ nw_b,
                                                         double* __restrict__ en_b,
                                                         uint16_t* __restrict__ fpos,
                                                         int32_t* __restrict__ fcnt, Ctl* ctl) {
    __shared__ Lds<W, V> L;
    __shared__ unsigned fl;
    if (wg_flags(ctl, &fl)) return;
    for (int b = blockIdx.x; b < sc.B; b += gridDim.x)
        annihilate_bucket<W, V, EXT>(sys, in, out, sc, rec2, soff, scur, rel, need_b, recs_b, nw_b, en_b, fpos, fcnt,
                                ctl, b, L);
}

// ---------------------------------------------------------------------------
// Diagonals H_jj - H_00 of the determinants that entered the store this step
// (molecular systems; lattice systems compute theirs in the per-bucket
// kernel).  Work item g covers buckets [g*span, (g+1)*span): h_pp, X and J
// are staged in LDS, then one lane per listed determinant sums its diagonal
// in the canonical order.  Done here rather than in the per-bucket kernel
// because each diagonal is a long serial chain that would hold that
// kernel's LDS hash table while one wave works.  The span grows with the
// bucket count (about 2048 work items, at most 32 buckets each) so that
// small stores still spread their diagonals over many workgroups.
// ---------------------------------------------------------------------------
constexpr int kFreshSpan = 32;  // largest span

__host__ __device__ inline int fresh_span(int B) {
    const int s = B / 2048;
    return s < 1 ? 1 : (s > kFreshSpan ? kFreshSpan : s);
}
__host__ __device__ inline int64_t fresh_items(int B) {
    const int s = fresh_span(B);
    return (B + s - 1) / s;
}

// h_pp, X and J (doubles), then each lane's occupied orbitals (one byte each,
// lane-interleaved) for the n_el electrons.
__host__ __device__ inline size_t fresh_lds_bytes(int N, int nel) {
    return sizeof(double) * ((size_t)N + 2 * (size_t)N * N) + (size_t)nel * kThreads;
}

// The diagonal of h_diag_tab (same terms, same order) from the determinant's
// occupied orbitals listed in LDS, alpha then beta, ascending: o[i * kThreads]
// is the i-th.  Each term is an index read, a table read and an add, where
// the bit-mask walk spent a dozen instructions finding the next orbital.
__device__ __forceinline__ double h_diag_list(const double* hd, const double* X, const double* J, int N, int na,
                                              int nb, const uint8_t* o) {
    const int n = na + nb;
    double acc = 0.0;
    // unrolled by four: the index and table reads of four terms are in
    // flight together, ahead of their (ordered) adds
#pragma unroll 4
    for (int i = 0; i < n; ++i) acc = acc + hd[o[i * kThreads]];
    for (int i = 0; i < na; ++i) {
        const int p = o[i * kThreads];
        const double* xr = X + p * N;
        const double* jr = J + p * N;
#pragma unroll 4
        for (int k = i + 1; k < na; ++k) acc = acc + xr[o[k * kThreads]];
#pragma unroll 4
        for (int k = na; k < n; ++k) acc = acc + jr[o[k * kThreads]];
    }
    for (int i = na; i < n; ++i) {
        const double* xr = X + o[i * kThreads] * N;
#pragma unroll 4
        for (int k = i + 1; k < n; ++k) acc = acc + xr[o[k * kThreads]];
    }
    return acc;
}

// With LISTS the lanes' orbital lists follow the tables in `tabs`
// (fresh_lds_bytes); without, the sums walk the bit masks (the persistent
// batch kernel, whose LDS would otherwise cost it a workgroup per CU).
template <int W, class V, bool LISTS = true>
__device__ __forceinline__ void fresh_item(const SysView& sys, const Store<V>& out, double h00, int R, int B,
                                           const uint16_t* __restrict__ fpos, const int32_t* __restrict__ fcnt,
                                           int64_t g, double* tabs, int* pre) {
    const int span = fresh_span(B);
    const int b0 = (int)(g * span);
    const int nb = min(span, B - b0);
    const int N = sys.N;
    double* hd = tabs;
    double* xt = tabs + N;
    double* jt = xt + N * N;
    uint8_t* occ = reinterpret_cast<uint8_t*>(jt + N * N) + threadIdx.x;
    for (int i = threadIdx.x; i < N * N; i += kThreads) { xt[i] = sys.X[i]; jt[i] = sys.J[i]; }
    for (int i = threadIdx.x; i < N; i += kThreads) hd[i] = sys.Hd[i];
    if (threadIdx.x < nb) pre[threadIdx.x + 1] = fcnt[b0 + threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) {
        pre[0] = 0;
        for (int k = 1; k <= nb; ++k) pre[k] += pre[k - 1];
    }
    __syncthreads();
    const int total = pre[nb];
    for (int t = threadIdx.x; t < total; t += kThreads) {
        int lo = 0, hi = nb;  // bucket k with pre[k] <= t < pre[k+1]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pre[mid] <= t) lo = mid; else hi = mid;
        }
        const int64_t base = (int64_t)(b0 + lo) * R;
        const int64_t e = base + fpos[base + (t - pre[lo])];
        const Key<W> key = load_key<W>(out.keys + e * W);
        double h;
        if constexpr (LISTS) {
            // every determinant of the store has na alpha and nb beta electrons
            int i = 0;
            for (uint64_t x = key_alpha<W>(key); x; x &= x - 1) occ[(i++) * kThreads] = (uint8_t)ctz64(x);
            for (uint64_t x = key_beta<W>(key); x; x &= x - 1) occ[(i++) * kThreads] = (uint8_t)ctz64(x);
            h = h_diag_list(hd, xt, jt, N, sys.na, sys.nb, occ);
        } else {
            h = h_diag_tab(hd, xt, jt, N, key_alpha<W>(key), key_beta<W>(key));
        }
        out.diag[e] = h - h00;
    }
    __syncthreads();
}

template <int W, class V>
__global__ __launch_bounds__(kThreads) void k_fresh(SysView sys, Store<V> out, StepScalars sc,
                                                    const uint16_t* __restrict__ fpos,
                                                    const int32_t* __restrict__ fcnt, const Ctl* ctl) {
    extern __shared__ double tabs[];
    __shared__ int pre[kFreshSpan + 1];
    __shared__ unsigned fl;
    if (wg_flags(ctl, &fl)) return;
    const int64_t items = fresh_items(sc.B);
    for (int64_t g = blockIdx.x; g < items; g += gridDim.x)
        fresh_item<W, V>(sys, out, sc.h00, sc.R, sc.B, fpos, fcnt, g, tabs, pre);
}



// Post work for many buckets, in three launches.  Phase a: workgroup g
// reduces buckets [g*kPostSpan, (g+1)*kPostSpan) to partial totals.  Phase b
// (one workgroup): prefix of the partials and the global sums.  Phase c:
// workgroup g writes the attempt and sub-slab offsets of its buckets.
constexpr int kPostSpan = 1024;

struct PostPart {
    int64_t att, chk, need, cnt, rec, mx;
    double nw, en;
};

__global__ __launch_bounds__(256) void k_post_a(const int64_t* __restrict__ batt,
                                                const int32_t* __restrict__ count,
                                                const double* __restrict__ nw_b,
                                                const double* __restrict__ en_b,
                                                const int64_t* __restrict__ need_b,
                                                const int64_t* __restrict__ recs_b, int B,
                                                PostPart* __restrict__ part, const Ctl* ctl) {
    if (ctl->flags) return;
    __shared__ int64_t sh[4];
    __shared__ double shd[8];
    __shared__ int64_t shm[4];
    const int g0 = blockIdx.x * kPostSpan;
    const int per = kPostSpan / 256;
    const int b0 = g0 + threadIdx.x * per, b1 = min(B, b0 + per);
    int64_t la = 0, lk = 0, ln = 0, c = 0, r = 0, mx = 0;
    double nw = 0.0, en = 0.0;
    for (int b = b0; b < b1; ++b) {
        la += batt[b];
        lk += chunks_of(batt[b]);
        ln += need_b[b];
        const int64_t cb = count[b];
        c += cb;
        r += recs_b[b];
        mx = max(mx, cb);
        nw = nw + nw_b[b];
        en = en + en_b[b];
    }
    int64_t ta, tk, tn, tcr;
    (void)block_excl_scan<256, int64_t>(la, ta, sh);
    (void)block_excl_scan<256, int64_t>(lk, tk, sh);
    (void)block_excl_scan<256, int64_t>(ln, tn, sh);
    (void)block_excl_scan<256, int64_t>((c << 32) | r, tcr, sh);
    nw = wave_sum(nw);
    en = wave_sum(en);
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, (int64_t)__shfl_xor(mx, o));
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) { shd[w] = nw; shd[4 + w] = en; shm[w] = mx; }
    __syncthreads();
    if (threadIdx.x == 0) {
        PostPart p;
        p.att = ta;
        p.chk = tk;
        p.need = tn;
        p.cnt = tcr >> 32;
        p.rec = tcr & 0xFFFFFFFFLL;
        p.mx = max(max(shm[0], shm[1]), max(shm[2], shm[3]));
        p.nw = ((shd[0] + shd[1]) + shd[2]) + shd[3];
        p.en = ((shd[4] + shd[5]) + shd[6]) + shd[7];
        part[blockIdx.x] = p;
    }
}

__global__ __launch_bounds__(256) void k_post_b(PostPart* __restrict__ part, int G, int B,
                                                int64_t* __restrict__ aoff, int64_t* __restrict__ soff,
                                                Ctl* ctl,
                                                Ctl* __restrict__ host) {
    if (ctl->flags) {
        if (threadIdx.x == 0) *host = *ctl;
        return;
    }
    __shared__ int64_t sh[4];
    // exclusive prefix of the partials (chunks, slab sizes), in place;
    // the attempt total
    const int per = (G + 255) / 256;
    const int g0 = threadIdx.x * per, g1 = min(G, g0 + per);
    int64_t la = 0, lk = 0, ln = 0;
    for (int g = g0; g < g1; ++g) { la += part[g].att; lk += part[g].chk; ln += part[g].need; }
    int64_t ta, tk, tn;
    (void)block_excl_scan<256, int64_t>(la, ta, sh);
    int64_t rk = block_excl_scan<256, int64_t>(lk, tk, sh);
    int64_t rn = block_excl_scan<256, int64_t>(ln, tn, sh);
    for (int g = g0; g < g1; ++g) {
        const int64_t k = part[g].chk, n = part[g].need;
        part[g].chk = rk;
        part[g].need = rn;
        rk += k;
        rn += n;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double nw = 0.0, en = 0.0;
        int64_t c = 0, r = 0, m = 0;
        for (int g = 0; g < G; ++g) {
            nw = nw + part[g].nw;
            en = en + part[g].en;
            c += part[g].cnt;
            r += part[g].rec;
            m = max(m, part[g].mx);
        }
        aoff[B] = tk;
        soff[(int64_t)B * kSub] = tn;
        ctl->nw = nw;
        ctl->enum_ = en;
        ctl->ndets = c;
        ctl->attempts = ta;
        ctl->chunks = tk;
        ctl->nrec_out = r;
        ctl->max_count = m;
        ctl->nref_out = ctl->nref;
        ctl->rec_need = tn;
        ctl->nrec = 0;
        ctl->nref = 0.0;
        *host = *ctl;
    }
}

__global__ __launch_bounds__(256) void k_post_c(const int64_t* __restrict__ batt,
                                                const int64_t* __restrict__ rel,
                                                const int64_t* __restrict__ need_b, int B,
                                                const PostPart* __restrict__ part,
                                                int64_t* __restrict__ aoff, int64_t* __restrict__ soff,
                                                uint64_t* __restrict__ scur,
                                                int64_t* __restrict__ cmap, int64_t cmap_cap, const Ctl* ctl) {
    if (ctl->flags) return;
    __shared__ int64_t sh[4];
    const int g0 = blockIdx.x * kPostSpan;
    const int per = kPostSpan / 256;
    const int b0 = g0 + threadIdx.x * per, b1 = min(B, b0 + per);
    int64_t lk = 0, ln = 0;
    for (int b = b0; b < b1; ++b) { lk += chunks_of(batt[b]); ln += need_b[b]; }
    int64_t tk, tn;
    int64_t rk = part[blockIdx.x].chk + block_excl_scan<256, int64_t>(lk, tk, sh);
    int64_t rn = part[blockIdx.x].need + block_excl_scan<256, int64_t>(ln, tn, sh);
    for (int b = b0; b < b1; ++b) {
        aoff[b] = rk;
        const int64_t nk = chunks_of(batt[b]);
        for (int64_t c = 0; c < nk && rk + c < cmap_cap; ++c) cmap[rk + c] = ((int64_t)b << 32) | c;
        rk += nk;
        int64_t r0 = rel[(int64_t)b * kSub];
        for (int j = 0; j < kSub; ++j) {
            const int64_t r1 = j + 1 < kSub ? rel[(int64_t)b * kSub + j + 1] : need_b[b];
            set_subslab(soff, scur, b, j, rn + r0, rn + r1);
            r0 = r1;
        }
        rn += need_b[b];
    }
}

// After an import the per-bucket kernel leaves the slabs alone; size the
// next step's slabs from the imported counts (cursor minus start).
__global__ void k_import_slabs(const uint64_t* __restrict__ scur, const int64_t* __restrict__ soff, int B,
                               int64_t* __restrict__ rel, int64_t* __restrict__ need_b) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    int64_t acc = 0;
    for (int j = 0; j < kSub; ++j) {
        const int64_t i = (int64_t)b * kSub + j;
        rel[i] = acc;
        acc += slab_size((int32_t)((uint32_t)scur[i] - (uint32_t)soff[i]));
    }
    need_b[b] = acc;
}

// Post work as its own launch (one workgroup).
__global__ __launch_bounds__(kPostThreads) void k_post(const int64_t* __restrict__ batt,
                                               const int32_t* __restrict__ count,
                                               const double* __restrict__ nw_b,
                                               const double* __restrict__ en_b, int B,
                                               int64_t* __restrict__ aoff,
                                               const int64_t* __restrict__ rel,
                                               const int64_t* __restrict__ need_b,
                                               const int64_t* __restrict__ recs_b,
                                               int64_t* __restrict__ soff, uint64_t* __restrict__ scur,
                                               int64_t* __restrict__ cmap,
                                               int64_t cmap_cap, Ctl* ctl, Ctl* __restrict__ host) {
    __shared__ int64_t sh[4 * kPostThreads / 64], shm[kPostThreads / 64];
    __shared__ double shd[2 * kPostThreads / 64];
    __shared__ unsigned shf;
    post_work<kPostThreads>(batt, count, nw_b, en_b, rel, need_b, recs_b, B, aoff, soff, scur, cmap, cmap_cap, ctl, host,
                            sh, shd, shm, &shf);
}

// The chunk map from the chunk prefix (when the map had to grow after the
// post work): cmap[aoff[b] + c] = b << 32 | c.
__global__ void k_chunk_map(const int64_t* __restrict__ aoff, int B, int64_t* __restrict__ cmap) {
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x)
        for (int64_t c = aoff[b]; c < aoff[b + 1]; ++c) cmap[c] = ((int64_t)b << 32) | (c - aoff[b]);
}

// Pack the heat-bath tables into 8-byte entries: 48-bit alias threshold and
// column from the construction (the exact thresholds stay beside them; the
// generator takes the drawn column's value from the integrals).
__global__ void k_pchb_pack(const double* __restrict__ p, const int* __restrict__ a, size_t n,
                            uint64_t* __restrict__ out) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = hb_pack(p[i], a[i]);
}

// ---------------------------------------------------------------------------
// Batched launches: many independent walker populations (instances, each with
// its own integrals, parameters and store) advance one step in shared
// launches.  Instance i owns the work items [first[i], first[i+1]) of a
// launch (spawn chunks, or buckets); a workgroup takes items blockIdx.x,
// blockIdx.x + gridDim.x, ... and finds each item's instance by binary search
// over the prefix.  Every instance's arithmetic is that of its own launch, so
// its trajectory does not depend on the company it keeps.
// ---------------------------------------------------------------------------
template <int W, class V> struct Inst {
    SysView sys;
    Store<V> in, out;
    StepScalars sc;
    Rec<W, V>* rec2;
    int64_t *soff, *rel, *need_b, *recs_b;
    uint64_t* scur;
    double *nw_b, *en_b;
    uint16_t* fpos;
    int32_t* fcnt;
    int64_t* cmap;
    int64_t cmap_cap;
    Ctl* ctl;
    int gen;   // excitation generator (FCIQMC_GEN_*)
};

__device__ __forceinline__ int owner_of(const int64_t* __restrict__ first, int k, int64_t g) {
    int lo = 0, hi = k;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (first[mid] <= g) lo = mid; else hi = mid;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

template <int W, class V, int GEN>
__global__ __launch_bounds__(kThreads) void k_spawn_batch(const Inst<W, V>* __restrict__ inst,
                                                          const int64_t* __restrict__ first, int k) {
    __shared__ int32_t smpre[kMaxR];
    const int64_t total = first[k];
    for (int64_t g = blockIdx.x; g < total; g += gridDim.x) {
        const int i = owner_of(first, k, g);
        const Inst<W, V>& I = inst[i];
        spawn_chunk<W, V, GEN, false>(I.sys, I.in, I.sc, I.rec2, I.scur, I.ctl, I.cmap, g - first[i], smpre,
                                      I.sys.J, I.sys.SK);
    }
}

template <int W, class V>
__global__ __launch_bounds__(kThreads, 6) void k_annihilate_batch(const Inst<W, V>* __restrict__ inst,
                                                               const int64_t* __restrict__ first, int k) {
    __shared__ Lds<W, V> L;
    __shared__ unsigned fl;
    const int64_t total = first[k];
    for (int64_t g = blockIdx.x; g < total; g += gridDim.x) {
        const int i = owner_of(first, k, g);
        const Inst<W, V>& I = inst[i];
        if (wg_flags(I.ctl, &fl)) continue;  // this instance replays its step alone
        annihilate_bucket<W, V, false>(I.sys, I.in, I.out, I.sc, I.rec2, I.soff, I.scur, I.rel, I.need_b, I.recs_b,
                                I.nw_b, I.en_b, I.fpos, I.fcnt, I.ctl, (int)(g - first[i]), L);
    }
}

// New diagonals of the molecular members (work items as in k_fresh).
template <int W, class V>
__global__ __launch_bounds__(kThreads) void k_fresh_batch(const Inst<W, V>* __restrict__ inst,
                                                          const int64_t* __restrict__ first, int k) {
    extern __shared__ double tabs[];
    __shared__ int pre[kFreshSpan + 1];
    __shared__ unsigned fl;
    const int64_t total = first[k];
    for (int64_t g = blockIdx.x; g < total; g += gridDim.x) {
        const int i = owner_of(first, k, g);
        const Inst<W, V>& I = inst[i];
        if (I.sys.onsite) continue;
        if (wg_flags(I.ctl, &fl)) continue;
        fresh_item<W, V>(I.sys, I.out, I.sc.h00, I.sc.R, I.sc.B, I.fpos, I.fcnt, g - first[i], tabs, pre);
    }
}

// Post work of instance blockIdx.x, then its step scalars written to
// ctl_out[blockIdx.x] in pinned host memory (no copy operation per step).
template <int W, class V>
__global__ __launch_bounds__(kPostThreads) void k_post_batch(const Inst<W, V>* __restrict__ inst,
                                                             Ctl* __restrict__ ctl_out) {
    __shared__ int64_t sh[4 * kPostThreads / 64], shm[kPostThreads / 64];
    __shared__ double shd[2 * kPostThreads / 64];
    __shared__ unsigned fl;
    const Inst<W, V>& I = inst[blockIdx.x];
    post_work<kPostThreads>(I.out.batt, I.out.count, I.nw_b, I.en_b, I.rel, I.need_b, I.recs_b, I.sc.B,
                            I.out.aoff, I.soff, I.scur, I.cmap, I.cmap_cap, I.ctl, ctl_out + blockIdx.x, sh, shd, shm,
                            &fl);
}

// ---------------------------------------------------------------------------
// The whole batched step in one cooperative launch: spawn, annihilation, new
// diagonals and post work of every member, with a grid-wide barrier between
// the phases (every workgroup of a cooperative launch is resident, so all of
// them reach each barrier).  Work items and their owners are those of the
// separate launches above, so each member's arithmetic is unchanged.
// ---------------------------------------------------------------------------
struct GridBar {
    unsigned count;  // workgroups arrived at the current barrier
    unsigned gen;    // barriers completed
    unsigned err;    // a wait ran out (the launch's results are void)
    unsigned pad;
};

constexpr unsigned kBarrierSpins = 1u << 21;  // ~4 s of s_sleep 64: far beyond any phase

// Grid barrier.  Every wave first waits until all its memory operations
// have completed (its stores have reached this XCD's L2); after the
// workgroup barrier the first thread alone releases at device scope (the
// L2 write-back covers the whole workgroup's stores), reads the generation
// (completed before the arrival is counted) and counts in; the last to
// arrive resets the count and advances the generation, which the others
// wait for with a bounded spin; the first thread then acquires at device
// scope (invalidating the caches the whole workgroup reads through) before
// the second workgroup barrier releases the other waves.  Returns false on
// every workgroup once any wait has run out.
__device__ __forceinline__ bool grid_barrier(GridBar* bar, unsigned* shok) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        bool ok = true;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned g = __hip_atomic_load(&bar->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_s_waitcnt(0);  // the generation is read before the arrival counts
        const unsigned arrived = __hip_atomic_fetch_add(&bar->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == gridDim.x - 1) {
            __hip_atomic_store(&bar->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_s_waitcnt(0);  // the reset lands before the generation moves
            __hip_atomic_fetch_add(&bar->gen, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            // the wait backs off (s_sleep 1, 2, 4 ... 64, about 1.7 us at
            // most) so that the early workgroups' polls do not crowd the
            // memory channel the late ones still use
            unsigned spins = 0, nap = 1;
            while (__hip_atomic_load(&bar->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                switch (nap) {
                    case 1: __builtin_amdgcn_s_sleep(1); break;
                    case 2: __builtin_amdgcn_s_sleep(2); break;
                    case 4: __builtin_amdgcn_s_sleep(4); break;
                    case 8: __builtin_amdgcn_s_sleep(8); break;
                    case 16: __builtin_amdgcn_s_sleep(16); break;
                    case 32: __builtin_amdgcn_s_sleep(32); break;
                    default: __builtin_amdgcn_s_sleep(64); break;
                }
                if (nap < 64) nap <<= 1;
                if (++spins > kBarrierSpins) {
                    __hip_atomic_fetch_or(&bar->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = false;
                    break;
                }
            }
        }
        if (__hip_atomic_load(&bar->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = false;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *shok = ok ? 1u : 0u;
    }
    __syncthreads();
    return *shok != 0;
}

// One spawn chunk of a member with the generator chosen at run time
// (GEN < 0) or fixed (GEN >= 0).
template <int W, class V, int GEN>
__device__ __forceinline__ void spawn_member_chunk(const Inst<W, V>& I, int64_t g, int32_t* smpre) {
    if constexpr (GEN >= 0) {
        spawn_chunk<W, V, GEN, false>(I.sys, I.in, I.sc, I.rec2, I.scur, I.ctl, I.cmap, g, smpre, I.sys.J,
                                      I.sys.SK);
    } else {
        switch (I.gen) {
            case 0: spawn_member_chunk<W, V, 0>(I, g, smpre); break;
            case 1: spawn_member_chunk<W, V, 1>(I, g, smpre); break;
            case 2: spawn_member_chunk<W, V, 2>(I, g, smpre); break;
            case 3: spawn_member_chunk<W, V, 3>(I, g, smpre); break;
            default: spawn_member_chunk<W, V, 4>(I, g, smpre); break;
        }
    }
}

template <int W, class V> union StepLds {
    int32_t smpre[kMaxR];
    Lds<W, V> L;
    struct {
        int64_t sh[4 * kThreads / 64];
        int64_t shm[kThreads / 64];
        double shd[2 * kThreads / 64];
    } post;
};

// cfirst, bfirst, ffirst: prefixes of spawn chunks, buckets and new-diagonal
// work items over the k members; ctl_out: the members' step scalars in
// pinned host memory.
template <int W, class V, int GEN>
__global__ __launch_bounds__(kThreads, 6) void k_batch_step(const Inst<W, V>* __restrict__ inst,
                                                         const int64_t* __restrict__ cfirst,
                                                         const int64_t* __restrict__ bfirst,
                                                         const int64_t* __restrict__ ffirst, int k, GridBar* bar,
                                                         Ctl* __restrict__ ctl_out) {
    __shared__ StepLds<W, V> U;
    __shared__ int pre[kFreshSpan + 1];
    __shared__ unsigned fl, ok;
    extern __shared__ double tabs[];
    // spawn
    for (int64_t g = blockIdx.x; g < cfirst[k]; g += gridDim.x) {
        const int i = owner_of(cfirst, k, g);
        spawn_member_chunk<W, V, GEN>(inst[i], g - cfirst[i], U.smpre);
    }
    if (!grid_barrier(bar, &ok)) return;
    // death, annihilation, compaction, estimator partials
    for (int64_t g = blockIdx.x; g < bfirst[k]; g += gridDim.x) {
        const int i = owner_of(bfirst, k, g);
        const Inst<W, V>& I = inst[i];
        if (wg_flags(I.ctl, &fl)) continue;  // this member replays its step alone
        annihilate_bucket<W, V, false>(I.sys, I.in, I.out, I.sc, I.rec2, I.soff, I.scur, I.rel, I.need_b,
                                       I.recs_b, I.nw_b, I.en_b, I.fpos, I.fcnt, I.ctl, (int)(g - bfirst[i]), U.L);
    }
    if (!grid_barrier(bar, &ok)) return;
    // diagonals of the members' new determinants (molecular systems)
    for (int64_t g = blockIdx.x; g < ffirst[k]; g += gridDim.x) {
        const int i = owner_of(ffirst, k, g);
        const Inst<W, V>& I = inst[i];
        if (I.sys.onsite) continue;
        if (wg_flags(I.ctl, &fl)) continue;
        fresh_item<W, V, false>(I.sys, I.out, I.sc.h00, I.sc.R, I.sc.B, I.fpos, I.fcnt, g - ffirst[i], tabs, pre);
    }
    if (!grid_barrier(bar, &ok)) return;
    // post work, one workgroup per member
    for (int i = blockIdx.x; i < k; i += gridDim.x) {
        const Inst<W, V>& I = inst[i];
        post_work<kThreads, 0>(I.out.batt, I.out.count, I.nw_b, I.en_b, I.rel, I.need_b, I.recs_b, I.sc.B,
                               I.out.aoff, I.soff, I.scur, I.cmap, I.cmap_cap, I.ctl, ctl_out + i, U.post.sh, U.post.shd,
                               U.post.shm, &fl);
    }
}

// Most populated determinant of a store: largest |C|, ties to the smallest
// (alpha, beta) pair; one candidate per workgroup (value, alpha, beta),
// reduced on the host.  The order of comparison makes the winner unique.
__device__ __forceinline__ bool more_populated(double v, uint64_t a, uint64_t b, double w, uint64_t c, uint64_t d) {
    if (v != w) return v > w;
    if (a != c) return a < c;
    return b < d;
}

template <int W, class V>
__global__ __launch_bounds__(kThreads) void k_most_populated(Store<V> st, int R, int B, double* __restrict__ bv,
                                                             uint64_t* __restrict__ bk) {
    __shared__ double sv[kThreads];
    __shared__ uint64_t sa[kThreads], sb[kThreads];
    double v = -1.0;
    uint64_t a = ~0ULL, b = ~0ULL;
    for (int bk_ = blockIdx.x; bk_ < B; bk_ += gridDim.x) {
        const int cnt = st.count[bk_];
        for (int e = threadIdx.x; e < cnt; e += kThreads) {
            const int64_t x = (int64_t)bk_ * R + e;
            const Key<W> key = load_key<W>(st.keys + x * W);
            const double av = vabs(st.vals[x]);
            const uint64_t ka = key_alpha<W>(key), kb = key_beta<W>(key);
            if (more_populated(av, ka, kb, v, a, b)) { v = av; a = ka; b = kb; }
        }
    }
    sv[threadIdx.x] = v;
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const int j = threadIdx.x + o;
            if (more_populated(sv[j], sa[j], sb[j], sv[threadIdx.x], sa[threadIdx.x], sb[threadIdx.x])) {
                sv[threadIdx.x] = sv[j];
                sa[threadIdx.x] = sa[j];
                sb[threadIdx.x] = sb[j];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        bv[blockIdx.x] = sv[0];
        bk[2 * blockIdx.x] = sa[0];
        bk[2 * blockIdx.x + 1] = sb[0];
    }
}

// Copy the store to flat arrays (offsets from a count scan).
template <int W, class V>
__global__ __launch_bounds__(kThreads) void k_extract(Store<V> st, int R, const int64_t* __restrict__ off,
                                                      uint64_t* __restrict__ keys,
                                                      double* __restrict__ vals, int B) {
    for (int b = blockIdx.x; b < B; b += gridDim.x) {
        const int cnt = st.count[b];
        const int64_t o = off[b];
        for (int e = threadIdx.x; e < cnt; e += kThreads) {
            const int64_t src = (int64_t)b * R + e;
            for (int w = 0; w < W; ++w) keys[(o + e) * W + w] = st.keys[src * W + w];
            vals[o + e] = (double)st.vals[src];
        }
    }
}

// Matrix elements for parity checks: out[i] = <D_j|H|D_i>.
__global__ void k_hij(SysView sys, const uint64_t* __restrict__ di, const uint64_t* __restrict__ dj,
                      long long n, double* __restrict__ out) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const uint64_t a1 = di[2 * i], b1 = di[2 * i + 1], a2 = dj[2 * i], b2 = dj[2 * i + 1];
        if (a1 == a2 && b1 == b2) out[i] = h_diag(sys, a1, b1);
        else out[i] = h_offdiag(sys, a1, b1, a2, b2);
    }
}

// J/K/U tables copied out of the packed integrals, the same-spin pair term
// X = J - K of the diagonal (one rounding, as in the diagonal's sum) and the
// Cauchy-Schwarz hole weights SK = sqrt(|K|) (correctly rounded square root).
__global__ void k_build_jk(SysView sys, double* J, double* K, double* X, double* U, double* Hd, double* SK) {
    const int N = sys.N;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N * N; i += gridDim.x * blockDim.x) {
        const int p = i / N, q = i % N;
        const double j = eri(sys, p, p, q, q);
        const double k = eri(sys, p, q, q, p);
        J[i] = j;
        K[i] = k;
        X[i] = j - k;
        SK[i] = sqrt(fabs(k));
        if (p == q) { U[p] = eri(sys, p, p, p, p); Hd[p] = sys.h1[i]; }
    }
}

// ---------------------------------------------------------------------------
// Adaptive shift (Sec. "Adaptive Shift", Eq. (as_fval)).  Between the spawn
// and the merge of a step: clear the per-entry sums, then per bucket look up
// each record's target among the bucket's entries at tau (an LDS table) and
// add its weight w = |H| / |H_jj - E_0| (E_0 the shift; capped at 1e6) to
// its non-initiator parent's sum of all weights, and, when the target is
// occupied (the spawn is accepted), to its sum of accepted weights.
// ---------------------------------------------------------------------------
template <class V>
__global__ __launch_bounds__(kThreads) void k_ada_zero(Store<V> in, int R, int B, int64_t* __restrict__ acc,
                                                       int64_t* __restrict__ all) {
    for (int b = blockIdx.x; b < B; b += gridDim.x) {
        const int cnt = in.count[b];
        for (int e = threadIdx.x; e < cnt; e += kThreads) {
            acc[(int64_t)b * R + e] = 0;
            all[(int64_t)b * R + e] = 0;
        }
    }
}

template <int W> struct AdaTable {
    uint64_t key0[2 * kMaxR];
    uint64_t key1[W == 2 ? 2 * kMaxR : 1];
    int32_t idx[2 * kMaxR];
};

template <int W, class V>
__global__ __launch_bounds__(kThreads) void k_ada_weights(SysView sys, Store<V> in, StepScalars sc,
                                                          const Rec<W, V>* __restrict__ rec2,
                                                          const int64_t* __restrict__ soff,
                                                          const uint64_t* __restrict__ scur, Ctl* ctl) {
    __shared__ AdaTable<W> T;
    for (int b = blockIdx.x; b < sc.B; b += gridDim.x) {
        const int64_t eb = (int64_t)b * sc.R;
        const int cnt = in.count[b];
        int nslots = kThreads;
        while (nslots < (cnt * 4) / 3 + 1 && nslots < 2 * kMaxR) nslots <<= 1;
        const uint64_t mask = (uint64_t)(nslots - 1);
        for (int i = threadIdx.x; i < nslots; i += kThreads) {
            T.key0[i] = kEmpty;
            if constexpr (W == 2) T.key1[i] = kEmpty;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < cnt; e += kThreads) {
            const Key<W> key = load_key<W>(in.keys + (eb + e) * W);
            const int s = lds_find<W>(T, key, key_hash<W>(key), mask, true);
            if (s < 0) { atomicOr(&ctl->flags, kFlagTable); continue; }
            T.idx[s] = e;
        }
        __syncthreads();
        int64_t cum[kSub + 1], lo[kSub];
        cum[0] = 0;
#pragma unroll
        for (int j = 0; j < kSub; ++j) {
            lo[j] = soff[(int64_t)b * kSub + j];
            cum[j + 1] = cum[j] + (int32_t)((uint32_t)scur[(int64_t)b * kSub + j] - (uint32_t)lo[j]);
        }
        for (int64_t q = threadIdx.x; q < cum[kSub]; q += kThreads) {
            int64_t src = 0;
#pragma unroll
            for (int j = 0; j < kSub; ++j)
                if (q >= cum[j] && q < cum[j + 1]) src = lo[j] + (q - cum[j]);
            const int64_t par = sc.rec_par[src];
            if (par < 0) continue;
            const Rec<W, V> x = rec2[src];
            Key<W> key;
#pragma unroll
            for (int w = 0; w < W; ++w) key.w[w] = x.k[w];
            const int s = lds_find<W>(T, key, key_hash<W>(key), mask, false);
            double dj;
            if (s >= 0) {
                dj = in.diag[eb + T.idx[s]];
            } else {
                const double hd = h_diag(sys, key_alpha<W>(key), key_beta<W>(key));
                dj = hd - sc.h00;
            }
            const double den = fabs(dj - sc.S);
            double w = den > 0.0 ? sc.rec_h[src] / den : 0.0;
            if (w > 1e6) w = 1e6;
            const long long qw = (long long)floor(w * kAdaScale + 0.5);
            atomicAdd((unsigned long long*)&sc.ada_all[par], (unsigned long long)qw);
            if (s >= 0) atomicAdd((unsigned long long*)&sc.ada_acc[par], (unsigned long long)qw);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Replica-pair PT2 correction (Sec. "Perturbative correction", Eq.
// (pt2_correction)).  A determinant's bucket is the top bits of its hash,
// so with power-of-two bucket counts B_r the bucket of a determinant in a
// layout of B_max buckets is b and in replica r's layout b >> (log2 B_max -
// log2 B_r): work item b of a launch over B_max buckets reads bucket
// b >> k_r of each replica and keeps only the entries that fall into b.
// This lets the two replicas hold different bucket counts (a store that
// grew during the step).  Per work item, replica 1's discarded weights are
// summed per target in an LDS table, probed with replica 2's, and
// S^1 S^2 / (E_0 - (H_jj - H_00)) is added over the targets both discarded.
// ---------------------------------------------------------------------------
constexpr int kPtSlots = 2048;
constexpr int kPtPassLoad = 768;   // distinct keys aimed at per pass (table load <= 3/8 on average)
template <int W> struct PtTable {
    uint64_t key0[kPtSlots];
    uint64_t key1[W == 2 ? kPtSlots : 1];
    double w1[kPtSlots];
    double w2[kPtSlots];
    int64_t sh[kThreads / 64];
    double shd[kThreads / 64];
    int full;
};

// Whether an entry of hash h read through a replica layout `shift` levels
// coarser than B_max belongs to work item b.
__device__ __forceinline__ bool in_item(uint64_t h, int shift, uint32_t Bmax, int b) {
    return shift == 0 || (int)bucket_of(h, Bmax) == b;
}

// Discarded-spawn sum of work item b (Eq. (pt2_correction) before the
// 1/dtau^2).  Replica 1's targets are split into P passes by bits 16..31 of
// their hash (bits that neither the bucket nor the LDS slot uses) so that a
// pass fits the table; P starts from the record count and doubles if a
// pass still fills the table.
template <int W, class V>
__device__ __forceinline__ void pt2_bucket(const SysView& sys, const Rec<W, V>* __restrict__ rej1,
                                           const int64_t* __restrict__ off1, const int32_t* __restrict__ cnt1,
                                           int sh1, const Rec<W, V>* __restrict__ rej2,
                                           const int64_t* __restrict__ off2, const int32_t* __restrict__ cnt2,
                                           int sh2, uint32_t Bmax, int b, double e0, double h00,
                                           double* __restrict__ part, unsigned* __restrict__ err, PtTable<W>& T) {
    const int b1 = b >> sh1, b2 = b >> sh2;
    const int n1 = cnt1[b1], n2 = cnt2[b2];
    const int64_t o1 = off1[b1], o2 = off2[b2];
    int P = 1;
    while ((int64_t)n1 > (int64_t)P * kPtPassLoad && P < (1 << 16)) P <<= 1;
    double acc = 0.0;
    for (;;) {
        int nslots = kThreads;
        const int want = P == 1 ? (n1 * 4) / 3 + 1 : kPtSlots;
        while (nslots < want && nslots < kPtSlots) nslots <<= 1;
        const uint64_t mask = (uint64_t)(nslots - 1);
        bool full = false;
        acc = 0.0;
        for (int pass = 0; pass < P && !full; ++pass) {
            for (int i = threadIdx.x; i < nslots; i += kThreads) {
                T.key0[i] = kEmpty;
                if constexpr (W == 2) T.key1[i] = kEmpty;
                T.w1[i] = 0.0;
                T.w2[i] = 0.0;
            }
            if (threadIdx.x == 0) T.full = 0;
            __syncthreads();
            for (int q = threadIdx.x; q < n1; q += kThreads) {
                const Rec<W, V> x = rej1[o1 + q];
                Key<W> key;
#pragma unroll
                for (int w = 0; w < W; ++w) key.w[w] = x.k[w];
                const uint64_t h = key_hash<W>(key);
                if (!in_item(h, sh1, Bmax, b) || (int)((h >> 16) & (uint64_t)(P - 1)) != pass) continue;
                const int s = lds_find<W>(T, key, h, mask, true);
                if (s == -2) { T.full = 1; continue; }
                if (s < 0) { atomicOr(err, 1u); continue; }
                lds_add<double>(&T.w1[s], (double)x.v);
            }
            __syncthreads();
            full = T.full != 0;
            if (!full) {
                for (int q = threadIdx.x; q < n2; q += kThreads) {
                    const Rec<W, V> x = rej2[o2 + q];
                    Key<W> key;
#pragma unroll
                    for (int w = 0; w < W; ++w) key.w[w] = x.k[w];
                    const uint64_t h = key_hash<W>(key);
                    if (!in_item(h, sh2, Bmax, b) || (int)((h >> 16) & (uint64_t)(P - 1)) != pass) continue;
                    const int s = lds_find<W>(T, key, h, mask, false);
                    if (s >= 0) lds_add<double>(&T.w2[s], (double)x.v);
                }
                __syncthreads();
                for (int i = threadIdx.x; i < nslots; i += kThreads) {
                    const double a = T.w1[i], c = T.w2[i];
                    if (T.key0[i] == kEmpty || a == 0.0 || c == 0.0) continue;
                    Key<W> key;
                    key.w[0] = T.key0[i];
                    if constexpr (W == 2) key.w[1] = T.key1[i];
                    const double hd = h_diag(sys, key_alpha<W>(key), key_beta<W>(key));
                    const double dj = hd - h00;
                    const double num = a * c;
                    const double den = e0 - dj;
                    const double x = num / den;
                    acc = acc + x;
                }
            }
            __syncthreads();
        }
        if (!full || P >= (1 << 16)) {
            if (full) atomicOr(err, 1u);
            break;
        }
        P <<= 1;
    }
    acc = wave_sum(acc);
    if (lane_id() == 0) T.shd[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[b] = ((T.shd[0] + T.shd[1]) + T.shd[2]) + T.shd[3];
    __syncthreads();
}

// Replica overlap sum_i C_i^1 C_i^2 over work item b: the first store's
// entries in an LDS table (at most R = 1024 of them), probed with the
// second's.
template <int W, class V>
__device__ __forceinline__ void overlap_bucket(const Store<V>& s1, int sh1, const Store<V>& s2, int sh2, int R,
                                               uint32_t Bmax, int b, double* __restrict__ part,
                                               unsigned* __restrict__ err, PtTable<W>& T) {
    const int b1 = b >> sh1, b2 = b >> sh2;
    const int n1 = s1.count[b1], n2 = s2.count[b2];
    int nslots = kThreads;
    while (nslots < (n1 * 4) / 3 + 1 && nslots < kPtSlots) nslots <<= 1;
    const uint64_t mask = (uint64_t)(nslots - 1);
    const int64_t e1 = (int64_t)b1 * R, e2 = (int64_t)b2 * R;
    for (int i = threadIdx.x; i < nslots; i += kThreads) {
        T.key0[i] = kEmpty;
        if constexpr (W == 2) T.key1[i] = kEmpty;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n1; e += kThreads) {
        const Key<W> key = load_key<W>(s1.keys + (e1 + e) * W);
        const uint64_t h = key_hash<W>(key);
        if (!in_item(h, sh1, Bmax, b)) continue;
        const int s = lds_find<W>(T, key, h, mask, true);
        if (s < 0) { atomicOr(err, 1u); continue; }
        T.w1[s] = (double)s1.vals[e1 + e];
    }
    __syncthreads();
    double acc = 0.0;
    for (int e = threadIdx.x; e < n2; e += kThreads) {
        const Key<W> key = load_key<W>(s2.keys + (e2 + e) * W);
        const uint64_t h = key_hash<W>(key);
        if (!in_item(h, sh2, Bmax, b)) continue;
        const int s = lds_find<W>(T, key, h, mask, false);
        if (s >= 0) {
            const double q = T.w1[s] * (double)s2.vals[e2 + e];
            acc = acc + q;
        }
    }
    acc = wave_sum(acc);
    if (lane_id() == 0) T.shd[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[b] = ((T.shd[0] + T.shd[1]) + T.shd[2]) + T.shd[3];
    __syncthreads();
}

// Both sums of a replica pair's step over B_max = max(B_1, B_2) work items
// (bucket counts are powers of two): the overlap of the populations the
// step started from into part_ovl, the discarded-spawn sum into part_pt2.
template <int W, class V>
__global__ __launch_bounds__(kThreads) void k_pair_sums(SysView sys, Store<V> s1, int sh1, Store<V> s2, int sh2,
                                                        int R, const Rec<W, V>* __restrict__ rej1,
                                                        const int64_t* __restrict__ off1,
                                                        const int32_t* __restrict__ cnt1,
                                                        const Rec<W, V>* __restrict__ rej2,
                                                        const int64_t* __restrict__ off2,
                                                        const int32_t* __restrict__ cnt2, int Bmax, double e0,
                                                        double h00, double* __restrict__ part_ovl,
                                                        double* __restrict__ part_pt2, unsigned* __restrict__ err) {
    __shared__ PtTable<W> T;
    for (int b = blockIdx.x; b < Bmax; b += gridDim.x) {
        overlap_bucket<W, V>(s1, sh1, s2, sh2, R, (uint32_t)Bmax, b, part_ovl, err, T);
        pt2_bucket<W, V>(sys, rej1, off1, cnt1, sh1, rej2, off2, cnt2, sh2, (uint32_t)Bmax, b, e0, h00, part_pt2,
                         err, T);
    }
}

// Sum of n per-bucket partials in a fixed order (one workgroup).
__device__ __forceinline__ double sum_parts(const double* __restrict__ part, int n, double* shd) {
    double acc = 0.0;
    const int per = (n + kThreads - 1) / kThreads;
    for (int i = threadIdx.x * per; i < min(n, (int)(threadIdx.x + 1) * per); ++i) acc = acc + part[i];
    acc = wave_sum(acc);
    if (lane_id() == 0) shd[threadIdx.x >> 6] = acc;
    __syncthreads();
    const double t = ((shd[0] + shd[1]) + shd[2]) + shd[3];
    __syncthreads();
    return t;
}

// The two sums of a pair's partials (overlap into out[1], PT2 into out[0]).
__global__ __launch_bounds__(kThreads) void k_sum2(const double* __restrict__ part_ovl,
                                                   const double* __restrict__ part_pt2, int n,
                                                   double* __restrict__ out) {
    __shared__ double shd[kThreads / 64];
    const double o = sum_parts(part_ovl, n, shd);
    const double q = sum_parts(part_pt2, n, shd);
    if (threadIdx.x == 0) { out[0] = q; out[1] = o; }
}

// ---------------------------------------------------------------------------
// Replica 2-RDM (Sec. "Density matrix sampling and pure expectation
// values", Eq. (FCI2RDM)) over spin-orbital pairs: canonical index so = spin * N + orbital, pair index
// P(k,l) = k(2K-k-1)/2 + l-k-1 for k < l (K = 2N), matrix G[P(k,l) M +
// P(m,n)] of M = K(K-1)/2 rows.  Per paired step: an open-addressing table
// of each replica's population at tau, the exact diagonal terms
// C_i^1 C_i^2 over determinants occupied in both, and for every excitation
// D_i -> D_j a replica generated, (C_i / (m_i p_gen)) C_j^other / 2 times
// <D_i|a+_k a+_l a_n a_m|D_j>.
// ---------------------------------------------------------------------------
template <int W> struct PopTable {
    uint64_t* keys;   // slots * W
    double* vals;
    int32_t* used;    // 0 empty, 1 claimed
    uint64_t mask;
};

// Insert every entry of a store (B buckets of R entries, count[b] used).
template <int W, class V>
__global__ __launch_bounds__(kThreads) void k_pop_table(Store<V> st, int R, int B, PopTable<W> T) {
    for (int b = blockIdx.x; b < B; b += gridDim.x) {
        const int cnt = st.count[b];
        for (int e = threadIdx.x; e < cnt; e += kThreads) {
            const int64_t x = (int64_t)b * R + e;
            const Key<W> key = load_key<W>(st.keys + x * W);
            uint64_t s = key_hash<W>(key) & T.mask;
            while (atomicCAS(&T.used[s], 0, 1) != 0) s = (s + 1) & T.mask;
            store_key<W>(T.keys + s * W, key);
            T.vals[s] = (double)st.vals[x];
        }
    }
}

template <int W> __device__ __forceinline__ double pop_lookup(const PopTable<W>& T, const Key<W>& key) {
    uint64_t s = key_hash<W>(key) & T.mask;
    for (;;) {
        if (T.used[s] == 0) return 0.0;
        if (key_eq<W>(load_key<W>(T.keys + s * W), key)) return T.vals[s];
        s = (s + 1) & T.mask;
    }
}

__device__ __forceinline__ int64_t rdm_pair(int K, int k, int l) {
    return (int64_t)k * (2 * K - k - 1) / 2 + (l - k - 1);
}
// canonical spin-orbital index of (spin, orbital)
__device__ __forceinline__ int so_index(int N, int sg, int p) { return sg * N + p; }

// Fermion sign of <D_i| a+_k a+_l a_n a_m |D_j> with D_i the result of the
// operators on D_j (a, b its masks): each operator, applied right to left,
// counts the occupied spin orbitals below it in the current string.
__device__ __forceinline__ int rdm_parity(uint64_t a, uint64_t b, int N, int k, int l, int m, int n) {
    uint64_t A = a, B = b;
    int par = below(A, B, m / N, m % N);
    clear_so(A, B, m / N, m % N);
    par += below(A, B, n / N, n % N);
    clear_so(A, B, n / N, n % N);
    par += below(A, B, l / N, l % N);
    set_so(A, B, l / N, l % N);
    par += below(A, B, k / N, k % N);
    return par & 1;
}

// Diagonal terms: for each determinant of the first population, C^1 C^2
// (C^2 from the second population's table) on Gamma_{kl,kl} for every
// occupied pair k < l; summed per workgroup in LDS (M doubles of dynamic
// shared memory), then added to G.
template <int W, class V>
__global__ __launch_bounds__(kThreads) void k_rdm_diag(Store<V> s1, int R, int B, PopTable<W> T2, int N,
                                                       double* __restrict__ G) {
    extern __shared__ double dg[];
    const int K = 2 * N;
    const int64_t M = (int64_t)K * (K - 1) / 2;
    for (int64_t i = threadIdx.x; i < M; i += kThreads) dg[i] = 0.0;
    __syncthreads();
    for (int bk = blockIdx.x; bk < B; bk += gridDim.x) {
        const int cnt = s1.count[bk];
        for (int e = threadIdx.x; e < cnt; e += kThreads) {
            const int64_t x = (int64_t)bk * R + e;
            const Key<W> key = load_key<W>(s1.keys + x * W);
            const double c2 = pop_lookup<W>(T2, key);
            const double q = (double)s1.vals[x] * c2;
            if (q == 0.0) continue;
            const uint64_t A = key_alpha<W>(key), Bm = key_beta<W>(key);
            // occupied spin orbitals in canonical order: alpha, then beta
            for (int sk = 0; sk < 2; ++sk)
                for (uint64_t xk = sk ? Bm : A; xk; xk &= xk - 1) {
                    const int k = so_index(N, sk, ctz64(xk));
                    for (int sl = sk; sl < 2; ++sl)
                        for (uint64_t xl = sl ? Bm : A; xl; xl &= xl - 1) {
                            const int l = so_index(N, sl, ctz64(xl));
                            if (l <= k) continue;
                            const int64_t P = rdm_pair(K, k, l);
                            lds_add<double>(&dg[P], q);
                        }
                }
        }
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < M; i += kThreads)
        if (dg[i] != 0.0) atomicAdd(&G[i * M + i], dg[i]);
}

// Off-diagonal terms from n generated excitations of one replica, the
// child's coefficient from the other replica's table.
template <int W>
__global__ __launch_bounds__(kThreads) void k_rdm_off(const RdmRec<W>* __restrict__ rec, int64_t n,
                                                      PopTable<W> To, int N, double* __restrict__ G) {
    const int K = 2 * N;
    const int64_t M = (int64_t)K * (K - 1) / 2;
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < n; q += (int64_t)gridDim.x * kThreads) {
        const RdmRec<W> r = rec[q];
        if (r.w == 0.0) continue;
        Key<W> pk, ck;
#pragma unroll
        for (int w = 0; w < W; ++w) { pk.w[w] = r.par[w]; ck.w[w] = r.chi[w]; }
        const double cj = pop_lookup<W>(To, ck);
        if (cj == 0.0) continue;
        const double w1 = r.w * cj;
        const double h = w1 * 0.5;
        // bra D_i = parent, ket D_j = child: a_m a_n remove c\p, a+_l a+_k add p\c
        const uint64_t pa = key_alpha<W>(pk), pb = key_beta<W>(pk);
        const uint64_t ca = key_alpha<W>(ck), cb = key_beta<W>(ck);
        const uint64_t ra = ca & ~pa, rb = cb & ~pb;   // in the ket only
        const uint64_t xa = pa & ~ca, xb = pb & ~cb;   // in the bra only
        const int nr = popc64(ra) + popc64(rb);
        int rm[2], ad[2], c = 0, d = 0;
        for (uint64_t t = ra; t; t &= t - 1) rm[c++] = so_index(N, 0, ctz64(t));
        for (uint64_t t = rb; t; t &= t - 1) rm[c++] = so_index(N, 1, ctz64(t));
        for (uint64_t t = xa; t; t &= t - 1) ad[d++] = so_index(N, 0, ctz64(t));
        for (uint64_t t = xb; t; t &= t - 1) ad[d++] = so_index(N, 1, ctz64(t));
        if (nr == 2) {
            const int m = rm[0], nn = rm[1], k = ad[0], l = ad[1];
            const int par = rdm_parity(ca, cb, N, k, l, m, nn);
            atomicAdd(&G[rdm_pair(K, k, l) * M + rdm_pair(K, m, nn)], par ? -h : h);
        } else if (nr == 1) {
            // promotions over the orbitals q occupied in both
            const uint64_t qa = pa & ca, qb = pb & cb;
            for (int sq = 0; sq < 2; ++sq)
                for (uint64_t t = sq ? qb : qa; t; t &= t - 1) {
                    const int qq = so_index(N, sq, ctz64(t));
                    const int m = rm[0] < qq ? rm[0] : qq, nn = rm[0] < qq ? qq : rm[0];
                    const int k = ad[0] < qq ? ad[0] : qq, l = ad[0] < qq ? qq : ad[0];
                    const int par = rdm_parity(ca, cb, N, k, l, m, nn);
                    atomicAdd(&G[rdm_pair(K, k, l) * M + rdm_pair(K, m, nn)], par ? -h : h);
                }
        }
    }
}

// ---------------------------------------------------------------------------
// Deterministic space set-up and its per-step product.
// ---------------------------------------------------------------------------
// Open-addressing table of the space's determinants (hidx preset to -1).
template <int W>
__global__ void k_core_hash(const uint64_t* __restrict__ keys, int64_t n, uint64_t* __restrict__ hkeys,
                            int32_t* __restrict__ hidx, uint64_t mask) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const Key<W> key = load_key<W>(keys + k * W);
        uint64_t s = key_hash<W>(key) & mask;
        while (atomicCAS(&hidx[s], -1, (int32_t)k) != -1) s = (s + 1) & mask;
        store_key<W>(hkeys + s * W, key);
    }
}

// H^D by removal keys.  Two distinct determinants of the space are connected
// (a single or a double excitation) exactly when, in one of five classes,
// taking electrons out of each leaves the same pair of strings:
//   0: equal alpha, beta single (one beta out)    1: equal alpha, beta double (two beta out)
//   2: equal beta, alpha single (one alpha out)   3: equal beta, alpha double (two alpha out)
//   4: alpha single and beta single (one of each out)
// and the strings left are the two determinants' intersection, so a
// connected pair shares exactly one key of exactly one class (its class
// test below rejects the pairs that share a key of a class not theirs).
// Each class is processed on its own: every (determinant, removal) entry is
// hashed into an open-addressing table of counts, entries whose key occurs
// twice or more are gathered into groups, and the pairs of each group are
// tested exactly (the strings themselves, not the hash) and evaluated.  The
// work is linear in the entries (at most C(n,2) per determinant and class)
// plus the pairs within groups, instead of quadratic in the space.
__device__ __forceinline__ int rk_removals(int c, int na, int nb) {
    switch (c) {
        case 0: return nb;
        case 1: return nb * (nb - 1) / 2;
        case 2: return na;
        case 3: return na * (na - 1) / 2;
        default: return na * nb;
    }
}

// Removal m of class c from (a, b): the strings left.
__device__ __forceinline__ void rk_removal(int c, uint64_t a, uint64_t b, int m, int nb, uint64_t& ra, uint64_t& rb) {
    ra = a;
    rb = b;
    int x, y;
    switch (c) {
        case 0: rb &= ~(1ULL << select64(b, m)); break;
        case 1:
            pair_decode((uint64_t)m, popc64(b), x, y);
            rb &= ~((1ULL << select64(b, x)) | (1ULL << select64(b, y)));
            break;
        case 2: ra &= ~(1ULL << select64(a, m)); break;
        case 3:
            pair_decode((uint64_t)m, popc64(a), x, y);
            ra &= ~((1ULL << select64(a, x)) | (1ULL << select64(a, y)));
            break;
        default:
            ra &= ~(1ULL << select64(a, m / nb));
            rb &= ~(1ULL << select64(b, m % nb));
            break;
    }
}

// The pair belongs to class c (given equal removal keys of that class).
__device__ __forceinline__ bool rk_class_pair(int c, uint64_t a1, uint64_t b1, uint64_t a2, uint64_t b2) {
    const int da = popc64(a1 ^ a2), db = popc64(b1 ^ b2);
    switch (c) {
        case 0: return da == 0 && db == 2;
        case 1: return da == 0 && db == 4;
        case 2: return db == 0 && da == 2;
        case 3: return db == 0 && da == 4;
        default: return da == 2 && db == 2;
    }
}

__device__ __forceinline__ uint64_t rk_hash(uint64_t ra, uint64_t rb) {
    uint64_t h = mix64(ra ^ mix64(rb + 0x2545F4914F6CDD1DULL));
    return h == kEmpty ? kEmpty - 2 : h;
}

struct RkPass {
    int cls, na, nb, part, nparts;
    int64_t n, m;        // determinants, removals per determinant
    uint64_t mask;       // table slots - 1
};

__device__ __forceinline__ bool rk_mine(const RkPass& P, uint64_t h) {
    return P.nparts == 1 || (int)((h >> 40) % (uint64_t)P.nparts) == P.part;
}

// Count the entries of this pass's keys (th preset to kEmpty, tc to 0).
template <int W>
__global__ void k_rk_count(const uint64_t* __restrict__ keys, RkPass P, uint64_t* __restrict__ th,
                           uint32_t* __restrict__ tc, unsigned* __restrict__ err) {
    const int64_t total = P.n * P.m;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = e / P.m;
        const Key<W> key = load_key<W>(keys + k * W);
        uint64_t ra, rb;
        rk_removal(P.cls, key_alpha<W>(key), key_beta<W>(key), (int)(e - k * P.m), P.nb, ra, rb);
        const uint64_t h = rk_hash(ra, rb);
        if (!rk_mine(P, h)) continue;
        uint64_t s = h & P.mask;
        for (uint64_t probe = 0;; ++probe) {
            if (probe > P.mask) { atomicOr(err, 1u); break; }
            const uint64_t old = atomicCAS((unsigned long long*)&th[s], kEmpty, h);
            if (old == kEmpty || old == h) { atomicAdd(&tc[s], 1u); break; }
            s = (s + 1) & P.mask;
        }
    }
}

// Groups: the slots counted twice or more get a group (index in tg, start
// and size), the others -1.
__global__ void k_rk_groups(const uint32_t* __restrict__ tc, uint64_t slots, int32_t* __restrict__ tg,
                            int64_t* __restrict__ gstart, uint32_t* __restrict__ gsize, int64_t gcap,
                            unsigned long long* __restrict__ totals, unsigned* __restrict__ err) {
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < slots; s += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t c = tc[s];
        int32_t g = -1;
        if (c >= 2) {
            const unsigned long long gi = atomicAdd(&totals[0], 1ULL);
            const unsigned long long st = atomicAdd(&totals[1], (unsigned long long)c);
            if ((int64_t)gi < gcap) {
                g = (int32_t)gi;
                gstart[gi] = (int64_t)st;
                gsize[gi] = c;
            } else {
                atomicOr(err, 2u);
            }
        }
        tg[s] = g;
    }
}

// Entries of grouped keys into their group's range of gm (k << 32 | m).
template <int W>
__global__ void k_rk_scatter(const uint64_t* __restrict__ keys, RkPass P, const uint64_t* __restrict__ th,
                             const int32_t* __restrict__ tg, const int64_t* __restrict__ gstart,
                             uint32_t* __restrict__ gfill, uint64_t* __restrict__ gm, int64_t gmcap) {
    const int64_t total = P.n * P.m;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = e / P.m;
        const Key<W> key = load_key<W>(keys + k * W);
        const int m = (int)(e - k * P.m);
        uint64_t ra, rb;
        rk_removal(P.cls, key_alpha<W>(key), key_beta<W>(key), m, P.nb, ra, rb);
        const uint64_t h = rk_hash(ra, rb);
        if (!rk_mine(P, h)) continue;
        uint64_t s = h & P.mask;
        for (uint64_t probe = 0; probe <= P.mask && th[s] != h; ++probe) s = (s + 1) & P.mask;
        if (th[s] != h) continue;  // counted above, so present; a table error is flagged there
        const int32_t g = tg[s];
        if (g < 0) continue;
        const int64_t pos = gstart[g] + (int64_t)atomicAdd(&gfill[g], 1u);
        if (pos < gmcap) gm[pos] = ((uint64_t)k << 32) | (uint32_t)m;
    }
}

// The pairs of each group, one wave per group: equal removal keys (the
// strings, exactly) and the class test make a connected pair, found once.
// Row x gets H_xy = <D_x|H|D_y> and row y gets H_yx, each where nonzero:
// counted into cnt (rowp == nullptr) or stored at the row's next place.
template <int W>
__global__ __launch_bounds__(256) void k_rk_pairs(SysView sys, const uint64_t* __restrict__ keys, RkPass P,
                                                  const int64_t* __restrict__ gstart,
                                                  const uint32_t* __restrict__ gsize, int64_t ngroups,
                                                  const uint64_t* __restrict__ gm,
                                                  unsigned long long* __restrict__ cnt,
                                                  const int64_t* __restrict__ rowp,
                                                  unsigned long long* __restrict__ rfill,
                                                  int32_t* __restrict__ col, double* __restrict__ val) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t g = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); g < ngroups; g += waves) {
        const int64_t L = gsize[g], g0 = gstart[g];
        for (int64_t x = 0; x + 1 < L; ++x) {
            // entry x is the wave's; its partners y > x are spread over the lanes
            const uint64_t ex = gm[g0 + x];
            const int64_t kx = (int64_t)(ex >> 32);
            const Key<W> Kx = load_key<W>(keys + kx * W);
            const uint64_t ax = key_alpha<W>(Kx), bx = key_beta<W>(Kx);
            uint64_t rax, rbx;
            rk_removal(P.cls, ax, bx, (int)(uint32_t)ex, P.nb, rax, rbx);
          for (int64_t y = x + 1 + lane_id(); y < L; y += 64) {
            const uint64_t ey = gm[g0 + y];
            const int64_t ky = (int64_t)(ey >> 32);
            if (kx == ky) continue;
            const Key<W> Ky = load_key<W>(keys + ky * W);
            const uint64_t ay = key_alpha<W>(Ky), by = key_beta<W>(Ky);
            uint64_t ray, rby;
            rk_removal(P.cls, ay, by, (int)(uint32_t)ey, P.nb, ray, rby);
            if (rax != ray || rbx != rby || !rk_class_pair(P.cls, ax, bx, ay, by)) continue;
            const double hxy = h_offdiag(sys, ay, by, ax, bx);
            const double hyx = h_offdiag(sys, ax, bx, ay, by);
            if (!rowp) {
                if (hxy != 0.0) atomicAdd(&cnt[kx], 1ULL);
                if (hyx != 0.0) atomicAdd(&cnt[ky], 1ULL);
            } else {
                // the counting sweep found the same pairs, so each row fills
                // exactly its count; the bound only guards the buffer
                if (hxy != 0.0) {
                    const int64_t p = rowp[kx] + (int64_t)atomicAdd(&rfill[kx], 1ULL);
                    if (p < rowp[kx + 1]) { col[p] = (int32_t)ky; val[p] = hxy; }
                }
                if (hyx != 0.0) {
                    const int64_t p = rowp[ky] + (int64_t)atomicAdd(&rfill[ky], 1ULL);
                    if (p < rowp[ky + 1]) { col[p] = (int32_t)kx; val[p] = hyx; }
                }
            }
          }
        }
    }
}

// H_kk - H_00 of the space's determinants (the same sum as the store's).
template <int W>
__global__ void k_core_diag(SysView sys, const uint64_t* __restrict__ keys, int64_t n, double h00,
                            double* __restrict__ cdiag) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const Key<W> key = load_key<W>(keys + k * W);
        const double h = h_diag(sys, key_alpha<W>(key), key_beta<W>(key));
        cdiag[k] = h - h00;
    }
}

// Mark the space's determinants in the store (tag the diagonal slot) and
// read their coefficients into c; a determinant not found is counted.
template <int W, class V>
__global__ void k_core_tag(Store<V> st, int R, int B, const uint64_t* __restrict__ keys, int64_t n,
                           double* __restrict__ c, unsigned long long* __restrict__ missing) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const Key<W> key = load_key<W>(keys + k * W);
        const int b = (int)bucket_of(key_hash<W>(key), (uint32_t)B);
        const int cnt = st.count[b];
        bool found = false;
        for (int e = 0; e < cnt; ++e) {
            const int64_t x = (int64_t)b * R + e;
            if (key_eq<W>(load_key<W>(st.keys + x * W), key)) {
                st.diag[x] = core_tag(k);
                c[k] = (double)st.vals[x];
                found = true;
                break;
            }
        }
        if (!found) atomicAdd(missing, 1ULL);
    }
}

// (P^D C)_k = (1 - dtau (H_kk - S)) C_k - dtau sum_{j != k} H_kj C_j, one
// wave per row (CSR), the row sum reduced across the wave in a fixed order.
__global__ __launch_bounds__(kThreads) void k_core_spmv(const int64_t* __restrict__ rowp,
                                                        const int32_t* __restrict__ col,
                                                        const double* __restrict__ val,
                                                        const double* __restrict__ cdiag,
                                                        const double* __restrict__ c, double* __restrict__ d,
                                                        int64_t n, double tau, double S) {
    const int64_t row = ((int64_t)blockIdx.x * kThreads + threadIdx.x) >> 6;
    if (row >= n) return;  // whole waves
    double acc = 0.0;
    for (int64_t q = rowp[row] + lane_id(); q < rowp[row + 1]; q += 64) {
        const double x = val[q] * c[col[q]];
        acc = acc + x;
    }
    acc = wave_sum(acc);
    if (lane_id() == 0) {
        const double t1 = cdiag[row] - S;
        const double t2 = tau * t1;
        const double f = 1.0 - t2;
        const double xv = f * c[row];
        const double y = tau * acc;
        d[row] = xv - y;
    }
}

// PCHB weights and alias tables, one thread per row (rows: opposite-spin
// (I,J) first, then same-spin I<J).  Weights per Eq. (hbs) over spatial
// orbitals; alias tables by Vose's construction with LIFO work lists filled
// in ascending column order.
__global__ void k_pchb_build(SysView sys, double* w_opp, double* p_opp, int* a_opp, double* s_opp,
                             double* w_same, double* p_same, int* a_same, double* s_same,
                             double* scaled_ws, int* small_ws, int* large_ws) {
    const int N = sys.N;
    const int NN = N * N, np = N * (N - 1) / 2;
    const int rows = NN + np;
    for (int row = blockIdx.x * blockDim.x + threadIdx.x; row < rows; row += gridDim.x * blockDim.x) {
        const bool opp = row < NN;
        const int K = opp ? NN : np;
        double* w;
        double* prob;
        int* alias;
        double sum = 0.0;
        if (opp) {
            const int I = row / N, J = row % N;
            w = w_opp + (size_t)row * NN; prob = p_opp + (size_t)row * NN; alias = a_opp + (size_t)row * NN;
            for (int A = 0; A < N; ++A)
                for (int B = 0; B < N; ++B) {
                    double x = fabs(eri(sys, A, I, B, J));
                    if (A == I || B == J) x = 0.0;
                    w[A * N + B] = x;
                    sum = sum + x;
                }
            s_opp[row] = sum;
        } else {
            const int ij = row - NN;
            int I = 0, J = 0;
            pair_decode((uint64_t)ij, N, I, J);
            w = w_same + (size_t)ij * np; prob = p_same + (size_t)ij * np; alias = a_same + (size_t)ij * np;
            int ab = 0;
            for (int A = 0; A < N; ++A)
                for (int B = A + 1; B < N; ++B, ++ab) {
                    const double d = eri(sys, A, I, B, J);
                    const double e = eri(sys, A, J, B, I);
                    const double v = d - e;
                    double x = fabs(v);
                    if (A == I || A == J || B == I || B == J) x = 0.0;
                    w[ab] = x;
                    sum = sum + x;
                }
            s_same[ij] = sum;
        }
        // private work lists: opposite-spin rows first, same-spin rows after them
        const size_t wb = opp ? (size_t)row * NN : (size_t)NN * NN + (size_t)(row - NN) * np;
        double* scaled = scaled_ws + wb;
        int* small = small_ws + wb;
        int* large = large_ws + wb;
        if (sum == 0.0) {
            for (int c = 0; c < K; ++c) { prob[c] = 0.0; alias[c] = c; }
            continue;
        }
        int ns = 0, nl = 0;
        for (int c = 0; c < K; ++c) {
            const double x = w[c] * (double)K;
            scaled[c] = x / sum;
            alias[c] = c;
            if (scaled[c] < 1.0) small[ns++] = c; else large[nl++] = c;
        }
        while (ns > 0 && nl > 0) {
            const int s_ = small[--ns];
            const int l = large[--nl];
            prob[s_] = scaled[s_];
            alias[s_] = l;
            const double t = scaled[l] + scaled[s_];
            scaled[l] = t - 1.0;
            if (scaled[l] < 1.0) small[ns++] = l; else large[nl++] = l;
        }
        while (nl > 0) { const int l = large[--nl]; prob[l] = 1.0; alias[l] = l; }
        while (ns > 0) { const int s_ = small[--ns]; prob[s_] = 1.0; alias[s_] = s_; }
    }
}

}  // namespace fq
