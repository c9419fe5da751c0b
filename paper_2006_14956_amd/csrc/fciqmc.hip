// Host side of libfciqmc: the C ABI declared in include/fciqmc.h.
//
// The host validates inputs, owns device memory, launches the kernels of
// kernels.hpp on the caller's HIP stream and performs the only scalar
// bookkeeping the method needs between steps: the shift update (Sec. I),
// which uses the natural logarithm and is therefore evaluated on the host,
// and the blocking analysis of the recorded estimators.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fciqmc.h"
#include "errors.hpp"
#include "kernels.hpp"

using namespace fq;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

}  // namespace

int fq_set_error(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

namespace {

#define HIP_OK(expr)                                                                           \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(FCIQMC_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                                   \
    } while (0)

#define CHECK(expr)              \
    do {                         \
        int rc_ = (expr);        \
        if (rc_ != 0) return rc_; \
    } while (0)

// Device allocation tracked against a byte budget.
struct Arena {
    int64_t bytes = 0;
    int64_t budget = 0;  // 0 = unlimited
    std::vector<void*> live;
    int alloc(void** p, size_t n) {
        n = std::max<size_t>(n, 256);
        if (budget > 0 && bytes + (int64_t)n > budget)
            return fail(FCIQMC_ENOMEM, "device memory budget exceeded (%lld + %zu > %lld bytes)",
                        (long long)bytes, n, (long long)budget);
        hipError_t e = hipMalloc(p, n);
        if (e != hipSuccess) {
            (void)hipGetLastError();  // the failure is reported here, not by a later launch check
            return fail(FCIQMC_ENOMEM, "hipMalloc(%zu) failed: %s", n, hipGetErrorString(e));
        }
        bytes += (int64_t)n;
        live.push_back(*p);
        sizes.push_back((int64_t)n);
        return 0;
    }
    void release(void* p) {
        if (!p) return;
        for (size_t i = 0; i < live.size(); ++i)
            if (live[i] == p) {
                (void)hipFree(p);
                bytes -= sizes[i];
                live.erase(live.begin() + i);
                sizes.erase(sizes.begin() + i);
                return;
            }
    }
    void clear() {
        for (void* p : live) (void)hipFree(p);
        live.clear();
        sizes.clear();
        bytes = 0;
    }
    std::vector<int64_t> sizes;
};

template <class T> int dalloc(Arena& a, T** p, size_t count) {
    return a.alloc(reinterpret_cast<void**>(p), count * sizeof(T));
}

constexpr int kGens = 5;  // FCIQMC_GEN_UNIFORM .. FCIQMC_GEN_PE

uint64_t next_pow2(uint64_t x) {
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace

// ---------------------------------------------------------------------------
// System: integrals and derived tables on the device.
// ---------------------------------------------------------------------------
struct fciqmc_system {
    int N = 0, na = 0, nb = 0;
    double e_core = 0.0;
    bool onsite = false;
    Arena arena;
    double *h1 = nullptr, *eri = nullptr, *J = nullptr, *K = nullptr, *X = nullptr, *U = nullptr, *Hd = nullptr,
           *SK = nullptr;
    int *deg = nullptr, *nbr = nullptr, *pair_of = nullptr;
    double *lat_pe = nullptr, *lat_pz = nullptr;
    bool pchb = false;
    std::vector<double> h1_host, eri_host;  // host copies (variational energy of an RDM)
    uint64_t *hb_opp = nullptr, *hb_same = nullptr;  // packed alias tables
    double *hbp_opp = nullptr, *hbp_same = nullptr;  // their exact thresholds
    double *hb_sum_opp = nullptr, *hb_sum_same = nullptr;  // their row sums
    int device = 0;

    SysView view() const {
        SysView v{};
        v.N = N; v.na = na; v.nb = nb; v.n = na + nb;
        v.onsite = onsite ? 1 : 0;
        v.h1 = h1; v.eri = eri; v.J = J; v.K = K; v.X = X; v.U = U; v.Hd = Hd; v.SK = SK;
        v.deg = deg; v.nbr = nbr;
        v.lat_pe = lat_pe; v.lat_pz = lat_pz;
        v.hb_opp = hb_opp;
        v.hb_same = hb_same;
        v.hbp_opp = hbp_opp;
        v.hbp_same = hbp_same;
        v.hb_sum_opp = hb_sum_opp;
        v.hb_sum_same = hb_sum_same;
        v.pair_of = pair_of;
        v.mN = N > 0 ? (uint32_t)(((1u << 20) + N - 1) / N) : 0u;
        v.mnb = nb > 0 ? (uint32_t)(((1u << 20) + nb - 1) / nb) : 0u;
        return v;
    }
    ~fciqmc_system() { arena.clear(); }
};

static int build_pchb(fciqmc_system* s, hipStream_t stream) {
    if (s->pchb) return 0;
    const int N = s->N, NN = N * N, np = N * (N - 1) / 2;
    const size_t ko = (size_t)NN * NN, ks = (size_t)np * np;
    // weights, alias columns (scratch), alias thresholds and row sums, then
    // the packed tables the generator reads; a column index must fit the
    // packed entry's alias field
    if (NN > (1 << kHbAliasBits)) return fail(FCIQMC_EINVAL, "heat-bath tables take at most %d columns", 1 << kHbAliasBits);
    Arena tmp;
    double *w_opp = nullptr, *w_same = nullptr;
    int *a_opp = nullptr, *a_same = nullptr;
    CHECK(dalloc(tmp, &w_opp, ko));
    CHECK(dalloc(tmp, &a_opp, ko));
    CHECK(dalloc(tmp, &w_same, ks + 1));
    CHECK(dalloc(tmp, &a_same, ks + 1));
    CHECK(dalloc(s->arena, &s->hbp_opp, ko));
    CHECK(dalloc(s->arena, &s->hbp_same, ks + 1));
    double *p_opp = s->hbp_opp, *p_same = s->hbp_same;
    CHECK(dalloc(s->arena, &s->hb_sum_opp, NN));
    CHECK(dalloc(s->arena, &s->hb_sum_same, np + 1));
    CHECK(dalloc(s->arena, &s->hb_opp, ko));
    CHECK(dalloc(s->arena, &s->hb_same, ks + 1));
    double* scaled = nullptr;
    int *small = nullptr, *large = nullptr;
    const size_t kw = ko + ks + 1;
    CHECK(dalloc(tmp, &scaled, kw));
    CHECK(dalloc(tmp, &small, kw));
    CHECK(dalloc(tmp, &large, kw));
    // the same-spin rows use their own offsets into the scratch after the opposite rows:
    // row r of K columns uses [r*K, (r+1)*K) of a region sized for its class
    SysView v = s->view();
    const int rows = NN + np;
    hipLaunchKernelGGL(k_pchb_build, dim3((rows + 63) / 64), dim3(64), 0, stream, v, w_opp, p_opp, a_opp,
                       s->hb_sum_opp, w_same, p_same, a_same, s->hb_sum_same, scaled, small, large);
    hipLaunchKernelGGL(k_pchb_pack, dim3(4096), dim3(256), 0, stream, (const double*)p_opp, (const int*)a_opp, ko,
                       s->hb_opp);
    if (np > 0)
        hipLaunchKernelGGL(k_pchb_pack, dim3(4096), dim3(256), 0, stream, (const double*)p_same, (const int*)a_same,
                           ks, s->hb_same);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(stream));
    tmp.clear();
    s->pchb = true;
    return 0;
}

// ---------------------------------------------------------------------------
// Engine: the device state of one walker population for a fixed determinant
// width W and value type V (int32 walker numbers or FP64 coefficients).
// ---------------------------------------------------------------------------
struct EngineBase {
    bool fixed_b = false;  // the caller fixed the bucket count: no growth by occupancy
    // A call failed after it had released device buffers it could not
    // allocate again (over the memory budget, or hipMalloc failed): the
    // population is gone and every later call on the run is refused.
    bool broken = false;
    int refuse_if_broken() const {
        return broken ? fail(FCIQMC_ESTATE,
                             "the run lost its device buffers in an earlier failed call (out of "
                             "memory); free it")
                      : 0;
    }
    virtual ~EngineBase() {}
    virtual int step_once(int64_t t, double S, Ctl& out, int& retries, int64_t& attempts) = 0;
    virtual int set_walkers(const uint64_t* dets, const double* vals, int64_t n) = 0;
    virtual int get_walkers(std::vector<uint64_t>& ab, std::vector<double>& vals) = 0;
    virtual int64_t attempts_next() const = 0;
    virtual double last_nw() const = 0;
    virtual int64_t bytes() const = 0;
    virtual int enable_profile() = 0;
    virtual void kernel_times(double* ms, int64_t* launches) const = 0;
    virtual int64_t buckets() const = 0;
    virtual int64_t spawn_capacity() const = 0;
    virtual void set_stream(hipStream_t s) = 0;
    virtual hipStream_t get_stream() const = 0;
    virtual int kind() const = 0;        // determinant width and value type, see kind_of
    virtual int64_t ndets() const = 0;   // occupied determinants after the last step
    virtual int rebucket(int buckets) = 0;
    // semi-stochastic deterministic space
    virtual int set_core(int64_t n_core) = 0;
    virtual int64_t core_size() const = 0;
    virtual int64_t core_nnz() const = 0;
    virtual const std::vector<uint64_t>& core_dets() const = 0;
    virtual int core_row(int64_t k, int32_t* cols, double* vals, int64_t cap, int64_t* n_out) = 0;
    // discarded spawns of each step, kept for a replica pair's PT2 correction
    virtual int set_collect(bool on) = 0;
    virtual void* rej_records() const = 0;
    virtual int64_t* rej_offsets() const = 0;
    virtual int32_t* rej_counts() const = 0;
    virtual const void* current_store() const = 0;  // Store<V> of the population
    virtual const void* previous_store() const = 0; // Store<V> the last step read (intact until the next merge)
    virtual int bucket_entries() const = 0;         // R
    // replica 2-RDM: every excitation of the last step (RdmRec<W>, rdm_count
    // attempt slots)
    virtual int set_rdm(bool on) = 0;
    // reference of the projected energy and initiator rule (the energy
    // zero H_00 is unchanged); the most populated determinant of the store
    virtual int set_reference(uint64_t a, uint64_t b) = 0;
    virtual int most_populated(uint64_t& a, uint64_t& b, double& v) = 0;
    virtual const void* rdm_records() const = 0;
    virtual int64_t rdm_count() const = 0;
};

// Largest deterministic space: H^D is built by testing all N_D^2 pairs.
constexpr int64_t kMaxCore = 1 << 23;
// Removal-key entries a pass of the H^D construction takes at most (its hash
// table has four slots per entry); a class with more entries is split into
// passes by the hash's bits.
constexpr int64_t kRkPerPass = 1 << 24;

// Engines of one kind share batched launches: 0 = (1 word, int32),
// 1 = (1 word, FP64), 2 = (2 words, int32), 3 = (2 words, FP64).
template <int W, class V> constexpr int kind_of() { return (W - 1) * 2 + (sizeof(V) == 8 ? 1 : 0); }

// kernels of one step, in launch order: spawn, annihilation, post
constexpr int kKernels = 3;
constexpr int64_t kProfileEvery = 16;
#ifndef FQ_OCCUPANCY
#define FQ_OCCUPANCY 1024
#endif
// determinants of the capacity hint per bucket of the walker store
constexpr int kBucketOccupancy = FQ_OCCUPANCY;
// mean occupied determinants per bucket above which the store doubles its
// bucket count after a step (the per-bucket hash tables stay below ~3/4 load)
constexpr int64_t kMaxMeanOccupancy = 600;

struct RunScalars {
    double tau, p_single, p_double, p_opp, n_a, c_min, h00;
    uint64_t seed, replica, ref_a, ref_b;
    int gen;
    int adaptive;  // adaptive shift for non-initiators
};

template <int W, class V> struct Engine : EngineBase {
    fciqmc_system* sys;
    hipStream_t stream;
    RunScalars rs;
    Arena arena;
    int B = 1, R = 1024;
    Store<V> st[2]{};
    int cur = 0;
    Rec<W, V>* rec = nullptr;   // staging of imported populations
    long long cap_stage = 0;
    Rec<W, V>* rec2 = nullptr;  // per-bucket record slabs
    long long cap = 0;
    long long rec_need = 0;     // slab capacity the next step reserves
    int32_t* scount = nullptr;  // records per sub-slab when slabs are rebuilt, B*kSub (zero between uses)
    int64_t* soff = nullptr;    // sub-slab offsets, B*kSub+1
    uint64_t* scur = nullptr;   // sub-slab cursor words (end << 32 | next place), B*kSub
    int64_t* rel = nullptr;     // next step's sub-slab offsets within their bucket, B*kSub
    int64_t* need_b = nullptr;  // next step's slab size per bucket, B
    int64_t* recs_b = nullptr;  // records per bucket this step, B
    PostPart* part = nullptr;   // partial totals of the multi-workgroup post work
    double *nw_b = nullptr, *en_b = nullptr;
    uint16_t* fpos = nullptr;   // per bucket: output positions of new determinants (molecular systems)
    int32_t* fcnt = nullptr;    // per bucket: their number
    Ctl* ctl = nullptr;
    Ctl* hctl = nullptr;  // pinned
    int64_t att_next = 0;
    int64_t chunk_next = 0;     // spawn chunks of the next step
    int64_t* cmap = nullptr;    // chunk -> bucket << 32 | local chunk, for the next step
    int64_t cap_cmap = 0;
    int64_t max_b = 1 << 22;
    bool dirty = false;  // a step stopped on a flag; counters need rebuilding
    // The spawn launch of step t+1 is queued right after step t's post work,
    // before the host reads step t's scalars (spawning does not use the
    // shift).  It is discarded and launched again if step t fails or a buffer
    // it used has to grow.
    bool pending = false;
    int64_t pending_t = -1;
    hipEvent_t ev_copy = nullptr;  // the step scalars have reached the host
    // optional per-kernel timing (HIP events around each launch of a step),
    // one set per step parity since the next spawn is queued early
    bool profile = false;
    // semi-stochastic deterministic space (Sec. "Semi-stochastic FCIQMC"):
    // its determinants ascending, H^D in CSR without the diagonal, the
    // diagonal H_kk - H_00, C_D for each store, and P^D C_D of the step
    int64_t ncore = 0, nnz = 0;
    std::vector<uint64_t> core_host;  // alpha, beta masks of each determinant
    uint64_t* core_keys = nullptr;
    uint64_t* core_hkeys = nullptr;
    int32_t* core_hidx = nullptr;
    uint64_t core_hmask = 0;
    double* core_cdiag = nullptr;
    double* core_cv[2] = {nullptr, nullptr};
    double* core_dv = nullptr;
    int64_t* core_rowp = nullptr;
    int32_t* core_col = nullptr;
    double* core_val = nullptr;
    unsigned long long* core_missing = nullptr;
    // discarded spawns of the last step (replica-pair PT2): records laid out
    // like the slabs, per-bucket start and count
    // adaptive shift: per record the non-initiator parent and |H| (laid out
    // like the slabs), per store entry the weight sums
    int64_t* rec_par = nullptr;
    double* rec_h = nullptr;
    int64_t* ada_acc = nullptr;
    int64_t* ada_all = nullptr;
    // the accumulators of the population's entries are zero: the merge that
    // produced it cleared them, and no weight pass has run on it since
    bool ada_clean = false;
    bool keep_rej = false;
    Rec<W, V>* rej = nullptr;
    long long cap_rej = 0;
    // replica 2-RDM sampling: one record per attempt slot of the last spawn
    bool rdm_on = false;
    RdmRec<W>* rdm = nullptr;
    int64_t cap_rdm = 0;
    int64_t rdm_n = 0;
    int64_t* rej_off = nullptr;
    int32_t* rej_cnt = nullptr;
    hipEvent_t ev[2][kKernels + 1]{};
    double kms[kKernels]{};
    int64_t klaunch = 0;

    Engine(fciqmc_system* s, hipStream_t st_, const RunScalars& r) : sys(s), stream(st_), rs(r) {}
    ~Engine() override {
        (void)hipStreamSynchronize(stream);
        arena.clear();
        if (hctl) (void)hipHostFree(hctl);
        if (ev_copy) (void)hipEventDestroy(ev_copy);
        if (profile)
            for (auto& set : ev)
                for (auto& e : set) (void)hipEventDestroy(e);
    }
    int enable_profile() override {
        if (profile) return 0;
        CHECK(discard_pending());  // the next spawn launch then carries its events
        for (auto& set : ev)
            for (auto& e : set) HIP_OK(hipEventCreate(&e));
        profile = true;
        return 0;
    }
    // Steps timed by events: one in kProfileEvery (event markers cost a few
    // microseconds each, comparable to a kernel at cache-resident sizes).
    static bool sampled(int64_t t) { return t % kProfileEvery == 0; }
    void mark(int set, int i) {
        if (profile && set >= 0) (void)hipEventRecord(ev[set][i], stream);
    }
    int collect(int set) {
        if (!profile || set < 0) return 0;
        for (int i = 0; i < kKernels; ++i) {
            float ms = 0.f;
            HIP_OK(hipEventElapsedTime(&ms, ev[set][i], ev[set][i + 1]));
            kms[i] += ms;
        }
        ++klaunch;
        return 0;
    }
    // Drop a queued spawn launch: wait for it, rewind the sub-slab cursors
    // and clear the step accumulators it touched (the slab offsets stay valid).
    int discard_pending() {
        if (!pending) return 0;
        HIP_OK(hipStreamSynchronize(stream));
        hipLaunchKernelGGL(k_slab_rewind, dim3((unsigned)std::min<int64_t>(4096, ((int64_t)B * kSub + 255) / 256)),
                           dim3(256), 0, stream, scur, (const int64_t*)soff, B * kSub);
        HIP_OK(hipGetLastError());
        HIP_OK(hipMemsetAsync(ctl, 0, offsetof(Ctl, nw), stream));
        pending = false;
        return 0;
    }
    int64_t bytes() const override { return arena.bytes; }
    void kernel_times(double* ms, int64_t* launches) const override {
        for (int i = 0; i < kKernels; ++i) ms[i] = kms[i];
        *launches = klaunch;
    }
    int64_t buckets() const override { return B; }
    int64_t spawn_capacity() const override { return cap; }
    int64_t attempts_next() const override { return att_next; }
    double last_nw() const override { return hctl ? hctl->nw : 0.0; }

    int alloc_store(Store<V>& s) {
        const size_t n = (size_t)B * R;
        CHECK(dalloc(arena, &s.keys, n * W));
        CHECK(dalloc(arena, &s.vals, n));
        CHECK(dalloc(arena, &s.diag, n));
        CHECK(dalloc(arena, &s.mpre, n));
        CHECK(dalloc(arena, &s.count, (size_t)B));
        CHECK(dalloc(arena, &s.batt, (size_t)B));
        CHECK(dalloc(arena, &s.aoff, (size_t)B + 1));
        HIP_OK(hipMemsetAsync(s.count, 0, sizeof(int32_t) * B, stream));
        HIP_OK(hipMemsetAsync(s.batt, 0, sizeof(int64_t) * B, stream));
        HIP_OK(hipMemsetAsync(s.aoff, 0, sizeof(int64_t) * (B + 1), stream));
        return 0;
    }
    void free_store(Store<V>& s) {
        arena.release(s.keys); arena.release(s.vals); arena.release(s.diag); arena.release(s.mpre);
        arena.release(s.count); arena.release(s.batt); arena.release(s.aoff);
        s = Store<V>{};
    }
    int alloc_buckets() {
        ada_clean = false;  // fresh accumulators hold no known values
        CHECK(alloc_store(st[0]));
        CHECK(alloc_store(st[1]));
        CHECK(dalloc(arena, &scount, (size_t)B * kSub));
        CHECK(dalloc(arena, &rel, (size_t)B * kSub));
        CHECK(dalloc(arena, &need_b, (size_t)B));
        CHECK(dalloc(arena, &recs_b, (size_t)B));
        CHECK(dalloc(arena, &part, (size_t)(B + kPostSpan - 1) / kPostSpan));
        CHECK(dalloc(arena, &soff, (size_t)B * kSub + 1));
        CHECK(dalloc(arena, &scur, (size_t)B * kSub));
        HIP_OK(hipMemsetAsync(scount, 0, sizeof(int32_t) * B * kSub, stream));
        HIP_OK(hipMemsetAsync(soff, 0, sizeof(int64_t) * (B * kSub + 1), stream));
        HIP_OK(hipMemsetAsync(scur, 0, sizeof(uint64_t) * B * kSub, stream));
        CHECK(dalloc(arena, &nw_b, (size_t)B));
        CHECK(dalloc(arena, &en_b, (size_t)B));
        if (!sys->onsite) {
            CHECK(dalloc(arena, &fpos, (size_t)B * R));
            CHECK(dalloc(arena, &fcnt, (size_t)B));
        }
        if (keep_rej) CHECK(alloc_rej_index());
        if (rs.adaptive) {
            CHECK(dalloc(arena, &ada_acc, (size_t)B * R));
            CHECK(dalloc(arena, &ada_all, (size_t)B * R));
        }
        return 0;
    }
    int alloc_rej_index() {
        CHECK(dalloc(arena, &rej_off, (size_t)B));
        CHECK(dalloc(arena, &rej_cnt, (size_t)B));
        HIP_OK(hipMemsetAsync(rej_off, 0, sizeof(int64_t) * B, stream));
        HIP_OK(hipMemsetAsync(rej_cnt, 0, sizeof(int32_t) * B, stream));
        return 0;
    }
    void free_buckets() {
        free_store(st[0]);
        free_store(st[1]);
        arena.release(scount); arena.release(soff); arena.release(scur);
        arena.release(rel); arena.release(need_b); arena.release(recs_b); arena.release(part);
        rel = nullptr; need_b = nullptr; recs_b = nullptr; part = nullptr;
        arena.release(rej_off); arena.release(rej_cnt);
        rej_off = nullptr; rej_cnt = nullptr;
        arena.release(ada_acc); arena.release(ada_all);
        ada_acc = nullptr; ada_all = nullptr;
        arena.release(nw_b); arena.release(en_b);
        arena.release(fpos); arena.release(fcnt);
        scount = nullptr; soff = nullptr; scur = nullptr; nw_b = en_b = nullptr;
        fpos = nullptr; fcnt = nullptr;
    }
    // Replace buffer p by one of n elements (contents are not kept): the new
    // one is allocated first and the old one kept if that fails; only when
    // the budget cannot hold both is the old one released first, and if the
    // allocation still fails the run is marked broken (p is then null).
    template <class T> int regrow(T*& p, size_t n) {
        T* q = nullptr;
        if (dalloc(arena, &q, n) == 0) {
            arena.release(p);
            p = q;
            return 0;
        }
        arena.release(p);
        p = nullptr;
        const int rc = dalloc(arena, &q, n);
        if (rc) {
            broken = true;
            return rc;
        }
        p = q;
        return 0;
    }
    // Grow the slab buffer to hold c records (contents are not kept).
    int ensure_slabs(long long c) {
        if (c <= cap) return 0;
        const long long nc = c + c / 4;
        CHECK(regrow(rec2, (size_t)nc));
        if (rs.adaptive) {
            CHECK(regrow(rec_par, (size_t)nc));
            CHECK(regrow(rec_h, (size_t)nc));
        }
        cap = nc;
        return cursor_range();
    }
    // Record places are 32-bit in the sub-slab cursor words: the slabs plus
    // two steps of attempts (a spawn queued behind a failed step counts on)
    // stay below 2^32, about 1.3e9 attempts per step.
    int cursor_range() const {
        if ((uint64_t)cap + 2ULL * (uint64_t)cap_cmap * kChunk >= (1ULL << 32))
            return fail(FCIQMC_EOVERFLOW, "%lld record places and %lld spawn chunks per step exceed the 32-bit "
                        "record cursors", (long long)cap, (long long)cap_cmap);
        return 0;
    }
    // The discarded-spawn buffer follows the slab capacity, but is replaced
    // only right before a merge: the records of the last accepted step stay
    // readable after it (a replica pair sums them then).
    int ensure_rej() {
        if (!keep_rej || cap_rej >= cap) return 0;
        HIP_OK(hipStreamSynchronize(stream));  // a queued pair sum may still read the records
        CHECK(regrow(rej, (size_t)cap));
        cap_rej = cap;
        return 0;
    }
    int ensure_stage(long long c) {
        if (c <= cap_stage) return 0;
        CHECK(regrow(rec, (size_t)c));
        cap_stage = c;
        return 0;
    }

    int init(int buckets, long long spawn_cap, int64_t budget) {
        arena.budget = budget;
        B = buckets;
        HIP_OK(hipHostMalloc((void**)&hctl, sizeof(Ctl), hipHostMallocCoherent));  // written by kernels
        HIP_OK(hipEventCreateWithFlags(&ev_copy, hipEventDisableTiming));
        CHECK(dalloc(arena, &ctl, 1));
        HIP_OK(hipMemsetAsync(ctl, 0, sizeof(Ctl), stream));
        CHECK(alloc_buckets());
        CHECK(ensure_slabs(spawn_cap));
        cap_cmap = std::max<int64_t>(1 << 16, spawn_cap / kChunk + 4 * (int64_t)B);
        CHECK(dalloc(arena, &cmap, (size_t)cap_cmap));
        return cursor_range();
    }
    // Room in the chunk map for the next step; after growth the map is
    // rebuilt from the chunk prefix the post work left in st[cur].
    int ensure_cmap() {
        chunk_next = hctl->chunks;
        if (chunk_next <= cap_cmap) return 0;
        const int64_t nc = chunk_next + chunk_next / 2 + 1024;
        CHECK(regrow(cmap, (size_t)nc));
        cap_cmap = nc;
        hipLaunchKernelGGL(k_chunk_map, dim3((unsigned)std::min<int64_t>((B + 255) / 256, 4096)), dim3(256), 0, stream,
                           st[cur].aoff, B, cmap);
        HIP_OK(hipGetLastError());
        return cursor_range();
    }

    StepScalars scalars(int64_t t, double S, int import_mode) const {
        StepScalars sc{};
        sc.t = t; sc.seed = rs.seed; sc.replica = rs.replica;
        sc.tau = rs.tau; sc.p_single = rs.p_single; sc.p_double = rs.p_double; sc.p_opp = rs.p_opp;
        {
            // the heat-bath generator's class factors, as it would form them per draw
            const double na = sys->na, nb = sys->nb;
            const double n_opp = na * nb;
            const double n_same = na * (na > 0 ? na - 1 : 0) / 2 + nb * (nb > 0 ? nb - 1 : 0) / 2;
            const double p1o = rs.p_double * rs.p_opp;
            const double p1s = rs.p_double * (1.0 - rs.p_opp);
            sc.p2_opp = n_opp > 0 ? p1o / n_opp : 0.0;
            sc.p2_same = n_same > 0 ? p1s / n_same : 0.0;
        }
        sc.n_a = rs.n_a; sc.c_min = rs.c_min; sc.S = S; sc.h00 = rs.h00;
        sc.ref_a = rs.ref_a; sc.ref_b = rs.ref_b;
        sc.B = B; sc.R = R; sc.spawn_cap = cap; sc.import_mode = import_mode;
        sc.ncore = ncore;
        if (ncore > 0) {
            sc.core_d = core_dv;
            sc.core_c = core_cv[1 - cur];
            sc.core_hkeys = core_hkeys;
            sc.core_hidx = core_hidx;
            sc.core_hmask = core_hmask;
        }
        if (keep_rej) {
            sc.rej = rej;
            sc.rej_off = rej_off;
            sc.rej_cnt = rej_cnt;
        }
        if (rs.adaptive) {
            sc.rec_par = rec_par;
            sc.rec_h = rec_h;
            sc.ada_acc = ada_acc;
            sc.ada_all = ada_all;
        }
        if (rdm_on) {
            sc.rdm_rec = rdm;
            sc.rdm_cap = cap_rdm;
        }
        return sc;
    }

    // Run the per-bucket kernel from st[cur] into st[1-cur] on the records in
    // the slabs, then the global sums; read the step's scalars back.
    int merge_and_post(const StepScalars& sc) {
        CHECK(launch_merge_post(sc, -1));
        HIP_OK(hipStreamSynchronize(stream));
        return 0;
    }

    // Queue annihilation, new diagonals and the post work of a step, which
    // writes the step scalars to the host (ev_copy marks its completion).
    int launch_merge_post(const StepScalars& sc, int set) {
        const SysView v = sys->view();
        Store<V> in = st[cur], out = st[1 - cur];
        const int gb = std::min(B, 32768);
        if (rs.adaptive && !sc.import_mode) {
            const unsigned ga = (unsigned)std::min(B, 8192);
            if (!ada_clean)
                hipLaunchKernelGGL((k_ada_zero<V>), dim3(ga), dim3(kThreads), 0, stream, in, R, B, ada_acc, ada_all);
            ada_clean = false;
            hipLaunchKernelGGL((k_ada_weights<W, V>), dim3(ga), dim3(kThreads), 0, stream, v, in, sc, rec2, soff,
                               scur, ctl);
        }
        if (ncore > 0 && !sc.import_mode)
            hipLaunchKernelGGL(k_core_spmv, dim3((unsigned)((ncore + 3) / 4)), dim3(kThreads), 0, stream, core_rowp,
                               core_col, core_val, core_cdiag, core_cv[cur], core_dv, ncore, rs.tau, sc.S);
        if (ext())
            hipLaunchKernelGGL((k_annihilate<W, V, true>), dim3(gb), dim3(kThreads), 0, stream, v, in, out, sc,
                               rec2, soff, scur, rel, need_b, recs_b, nw_b, en_b, fpos, fcnt, ctl);
        else
            hipLaunchKernelGGL((k_annihilate<W, V, false>), dim3(gb), dim3(kThreads), 0, stream, v, in, out, sc,
                               rec2, soff, scur, rel, need_b, recs_b, nw_b, en_b, fpos, fcnt, ctl);
        if (!sys->onsite) {
            const int64_t items = fresh_items(B);
            hipLaunchKernelGGL((k_fresh<W, V>), dim3((unsigned)std::min<int64_t>(items, 4096)), dim3(kThreads),
                               fresh_lds_bytes(sys->N, v.na + v.nb), stream, v, out, sc, fpos, fcnt, ctl);
        }
        mark(set, 2);
        if (sc.import_mode) {
            // slabs of the first step after an import: from the imported counts
            hipLaunchKernelGGL(k_import_slabs, dim3((B + 255) / 256), dim3(256), 0, stream, scur, soff, B, rel,
                               need_b);
        }
        if (B <= 4 * kPostSpan) {
            hipLaunchKernelGGL(k_post, dim3(1), dim3(kPostThreads), 0, stream, out.batt, out.count, nw_b, en_b,
                               B, out.aoff, rel, need_b, recs_b, soff, scur, cmap, cap_cmap, ctl, hctl);
        } else {
            const int G = (B + kPostSpan - 1) / kPostSpan;
            hipLaunchKernelGGL(k_post_a, dim3(G), dim3(256), 0, stream, out.batt, out.count, nw_b, en_b, need_b,
                               recs_b, B, part, ctl);
            hipLaunchKernelGGL(k_post_b, dim3(1), dim3(256), 0, stream, part, G, B, out.aoff, soff, ctl, hctl);
            hipLaunchKernelGGL(k_post_c, dim3(G), dim3(256), 0, stream, out.batt, rel, need_b, B, part, out.aoff,
                               soff, scur, cmap, cap_cmap, ctl);
        }
        mark(set, 3);
        HIP_OK(hipGetLastError());
        // the post kernel has written the step scalars to hctl (pinned host memory)
        HIP_OK(hipEventRecord(ev_copy, stream));
        return 0;
    }

    // After a step that stopped on a flag: clear the per-step accumulators and
    // rebuild the slabs from the counts the stopped step reached (the exact
    // record numbers per sub-slab, from its cursor), which leaves scount zero
    // again.
    int recover() {
        HIP_OK(hipMemsetAsync(ctl, 0, offsetof(Ctl, nw), stream));
        hipLaunchKernelGGL(k_slab_counts, dim3((unsigned)std::min<int64_t>(4096, ((int64_t)B * kSub + 255) / 256)),
                           dim3(256), 0, stream, (const uint64_t*)scur, (const int64_t*)soff, B * kSub, scount);
        hipLaunchKernelGGL(k_offsets, dim3(1), dim3(1024), 0, stream, scount, B * kSub, 1, soff, scur, ctl);
        HIP_OK(hipGetLastError());
        HIP_OK(hipMemcpyAsync(hctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
        HIP_OK(hipStreamSynchronize(stream));
        rec_need = hctl->rec_need;
        return ensure_slabs(rec_need);
    }

    int grow_buckets() {
        if ((int64_t)B * 2 > max_b) return fail(FCIQMC_EOVERFLOW, "walker store cannot grow beyond %d buckets", B);
        std::vector<uint64_t> ab;
        std::vector<double> vals;
        CHECK(get_walkers(ab, vals));
        broken = true;  // until the population is back in the new store
        free_buckets();
        B *= 2;
        CHECK(alloc_buckets());
        cur = 0;
        return import(ab.data(), vals.data(), (int64_t)vals.size());
    }

    // Load a population through the per-bucket merge with death and rounding off.
    int import(const uint64_t* ab, const double* vals, int64_t n) {
        CHECK(discard_pending());
        broken = true;  // until the population is in the store
        for (int attempt = 0; attempt < 24; ++attempt) {
            CHECK(ensure_stage(std::max<int64_t>(n, 1)));
            CHECK(ensure_slabs(std::max<int64_t>(n, 1)));
            std::vector<Rec<W, V>> h((size_t)std::max<int64_t>(n, 1));
            for (int64_t i = 0; i < n; ++i) {
                const uint64_t a = ab[2 * i], b = ab[2 * i + 1];
                if constexpr (W == 1) h[i].k[0] = a | (b << 32);
                else { h[i].k[0] = a; h[i].k[W - 1] = b; }
                h[i].v = (V)vals[i];
                h[i].flag = 1u;
            }
            if (n > 0)
                HIP_OK(hipMemcpyAsync(rec, h.data(), sizeof(Rec<W, V>) * n, hipMemcpyHostToDevice, stream));
            Ctl c{};
            c.nrec = (unsigned long long)n;
            HIP_OK(hipMemcpyAsync(ctl, &c, sizeof(Ctl), hipMemcpyHostToDevice, stream));
            HIP_OK(hipMemsetAsync(scount, 0, sizeof(int32_t) * B * kSub, stream));
            const unsigned gs = (unsigned)std::max<long long>(1, std::min<long long>(1024, (n + 255) / 256));
            if (n > 0)
                hipLaunchKernelGGL((k_bucketize<W, V>), dim3(gs), dim3(kThreads), 0, stream, rec, (long long)n, B,
                                   scount);
            hipLaunchKernelGGL(k_offsets, dim3(1), dim3(1024), 0, stream, scount, B * kSub, 0, soff, scur, ctl);
            if (n > 0)
                hipLaunchKernelGGL((k_scatter<W, V>), dim3(gs), dim3(kThreads), 0, stream, rec, (long long)n, B, rec2,
                                   scur);
            HIP_OK(hipGetLastError());
            StepScalars sc = scalars(0, 0.0, 1);
            CHECK(merge_and_post(sc));
            const unsigned flags = hctl->flags;
            if (flags == 0) {
                cur = 1 - cur;
                ada_clean = true;
                att_next = hctl->attempts;
                rec_need = hctl->rec_need;
                CHECK(ensure_cmap());
                CHECK(ensure_slabs(rec_need));
                broken = false;
                return tag_core();
            }
            if (flags & (kFlagTable | kFlagStore)) {
                if ((int64_t)B * 2 > max_b) return fail(FCIQMC_EOVERFLOW, "population does not fit the walker store");
                free_buckets();
                B *= 2;
                CHECK(alloc_buckets());
                cur = 0;
                continue;
            }
            return fail(FCIQMC_EDEVICE, "population import failed (device flags 0x%x)", flags);
        }
        return fail(FCIQMC_EOVERFLOW, "population import did not converge");
    }

    int set_walkers(const uint64_t* ab, const double* vals, int64_t n) override {
        CHECK(refuse_if_broken());
        clear_core();  // a new population has no deterministic space
        cur = 0;
        dirty = false;
        return import(ab, vals, n);
    }

    // ---- deterministic space ----
    void clear_core() {
        for (void* p : {(void*)core_keys, (void*)core_hkeys, (void*)core_hidx, (void*)core_cdiag, (void*)core_cv[0],
                        (void*)core_cv[1], (void*)core_dv, (void*)core_rowp, (void*)core_col, (void*)core_val,
                        (void*)core_missing})
            arena.release(p);
        core_keys = core_hkeys = nullptr;
        core_hidx = core_col = nullptr;
        core_cdiag = core_cv[0] = core_cv[1] = core_dv = core_val = nullptr;
        core_rowp = nullptr;
        core_missing = nullptr;
        core_host.clear();
        ncore = nnz = 0;
    }
    // Tag the space's determinants in the current store and read C_D.
    int tag_core() {
        if (ncore == 0) return 0;
        HIP_OK(hipMemsetAsync(core_missing, 0, sizeof(unsigned long long), stream));
        const unsigned g = (unsigned)std::min<int64_t>((ncore + 255) / 256, 4096);
        hipLaunchKernelGGL((k_core_tag<W, V>), dim3(g), dim3(256), 0, stream, st[cur], R, B, core_keys, ncore,
                           core_cv[cur], core_missing);
        HIP_OK(hipGetLastError());
        unsigned long long miss = 0;
        HIP_OK(hipMemcpyAsync(&miss, core_missing, sizeof(miss), hipMemcpyDeviceToHost, stream));
        HIP_OK(hipStreamSynchronize(stream));
        if (miss)
            return fail(FCIQMC_EDEVICE, "%llu determinants of the deterministic space are not in the population", miss);
        return 0;
    }
    // The n_core determinants of largest |C| (ties: ascending determinant),
    // H^D between them, and the tags in the store.
    int set_core(int64_t n_core) override {
        CHECK(refuse_if_broken());
        CHECK(discard_pending());  // a queued spawn ignores the new space
        clear_core();
        if (n_core == 0) return 0;
        std::vector<uint64_t> ab;
        std::vector<double> vals;
        CHECK(get_walkers(ab, vals));
        const int64_t n = (int64_t)vals.size();
        const int64_t nc = std::min(n_core, n);
        if (nc == 0) return 0;
        std::vector<int64_t> ord((size_t)n);
        for (int64_t i = 0; i < n; ++i) ord[(size_t)i] = i;
        // the nc first under a strict total order (a selection, linear in n)
        auto before = [&](int64_t x, int64_t y) {
            const double ax = std::fabs(vals[(size_t)x]), ay = std::fabs(vals[(size_t)y]);
            if (ax != ay) return ax > ay;
            if (ab[2 * x] != ab[2 * y]) return ab[2 * x] < ab[2 * y];
            return ab[2 * x + 1] < ab[2 * y + 1];
        };
        if (nc < n) std::nth_element(ord.begin(), ord.begin() + nc, ord.end(), before);
        std::vector<std::pair<uint64_t, uint64_t>> dets((size_t)nc);
        for (int64_t k = 0; k < nc; ++k) dets[(size_t)k] = {ab[2 * ord[(size_t)k]], ab[2 * ord[(size_t)k] + 1]};
        std::sort(dets.begin(), dets.end());
        core_host.resize((size_t)nc * 2);
        std::vector<uint64_t> keys((size_t)nc * W);
        for (int64_t k = 0; k < nc; ++k) {
            const uint64_t a = dets[(size_t)k].first, b = dets[(size_t)k].second;
            core_host[(size_t)(2 * k)] = a;
            core_host[(size_t)(2 * k + 1)] = b;
            if constexpr (W == 1) keys[(size_t)k] = a | (b << 32);
            else { keys[(size_t)(2 * k)] = a; keys[(size_t)(2 * k + 1)] = b; }
        }
        const int64_t slots = (int64_t)next_pow2((uint64_t)std::max<int64_t>(64, 2 * nc));
        CHECK(dalloc(arena, &core_keys, (size_t)nc * W));
        CHECK(dalloc(arena, &core_hkeys, (size_t)slots * W));
        CHECK(dalloc(arena, &core_hidx, (size_t)slots));
        CHECK(dalloc(arena, &core_cdiag, (size_t)nc));
        CHECK(dalloc(arena, &core_cv[0], (size_t)nc));
        CHECK(dalloc(arena, &core_cv[1], (size_t)nc));
        CHECK(dalloc(arena, &core_dv, (size_t)nc));
        CHECK(dalloc(arena, &core_rowp, (size_t)nc + 1));
        CHECK(dalloc(arena, &core_missing, 1));
        core_hmask = (uint64_t)slots - 1;
        HIP_OK(hipMemcpyAsync(core_keys, keys.data(), sizeof(uint64_t) * keys.size(), hipMemcpyHostToDevice, stream));
        HIP_OK(hipMemsetAsync(core_hidx, 0xFF, sizeof(int32_t) * slots, stream));
        const SysView v = sys->view();
        const unsigned g = (unsigned)std::min<int64_t>((nc + 255) / 256, 4096);
        hipLaunchKernelGGL((k_core_hash<W>), dim3(g), dim3(256), 0, stream, core_keys, nc, core_hkeys, core_hidx,
                           core_hmask);
        hipLaunchKernelGGL((k_core_diag<W>), dim3(g), dim3(256), 0, stream, v, core_keys, nc, rs.h00, core_cdiag);
        CHECK(build_hd(nc));
        ncore = nc;
        return tag_core();
    }
    // H^D between the space's determinants, by removal keys: for each of the
    // five classes (and hash partition), count the keys, gather the repeated
    // ones into groups and test their pairs; a counting sweep gives the row
    // sizes, their prefix on the host the row starts, and a filling sweep the
    // entries (a row's order is the order its pairs were found in).
    int build_hd(int64_t nc) {
        const SysView v = sys->view();
        const int na = v.na, nb = v.nb;
        auto removals = [&](int c) -> int64_t {
            switch (c) {
                case 0: return nb;
                case 1: return (int64_t)nb * (nb - 1) / 2;
                case 2: return na;
                case 3: return (int64_t)na * (na - 1) / 2;
                default: return (int64_t)na * nb;
            }
        };
        Arena tmp;
        struct Release {
            Arena& a;
            hipStream_t s;
            ~Release() { (void)hipStreamSynchronize(s); a.clear(); }
        } release{tmp, stream};
        unsigned long long *cnt = nullptr, *rfill = nullptr, *totals = nullptr;
        unsigned* err = nullptr;
        CHECK(dalloc(tmp, &cnt, (size_t)nc));
        CHECK(dalloc(tmp, &rfill, (size_t)nc));
        CHECK(dalloc(tmp, &totals, 2));
        CHECK(dalloc(tmp, &err, 1));
        HIP_OK(hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * nc, stream));
        HIP_OK(hipMemsetAsync(rfill, 0, sizeof(unsigned long long) * nc, stream));
        HIP_OK(hipMemsetAsync(err, 0, sizeof(unsigned), stream));
        int64_t emax = 0;
        for (int c = 0; c < 5; ++c) emax = std::max(emax, nc * removals(c));
        const int64_t per = std::min(emax, kRkPerPass);
        const int64_t slots = (int64_t)next_pow2((uint64_t)(4 * per + 64));
        uint64_t* th = nullptr;
        uint32_t *tc = nullptr, *gsize = nullptr, *gfill = nullptr;
        int32_t* tg = nullptr;
        int64_t* gstart = nullptr;
        uint64_t* gm = nullptr;
        int64_t gcap = per + 64, gmcap = 2 * per + 64;
        CHECK(dalloc(tmp, &th, (size_t)slots));
        CHECK(dalloc(tmp, &tc, (size_t)slots));
        CHECK(dalloc(tmp, &tg, (size_t)slots));
        CHECK(dalloc(tmp, &gstart, (size_t)gcap));
        CHECK(dalloc(tmp, &gsize, (size_t)gcap));
        CHECK(dalloc(tmp, &gfill, (size_t)gcap));
        CHECK(dalloc(tmp, &gm, (size_t)gmcap));
        int64_t* rowp_h = nullptr;
        std::vector<int64_t> rp((size_t)nc + 1, 0);
        for (int sweep = 0; sweep < 2; ++sweep) {
            if (sweep == 1) {
                std::vector<unsigned long long> hc((size_t)nc);
                HIP_OK(hipMemcpyAsync(hc.data(), cnt, sizeof(unsigned long long) * nc, hipMemcpyDeviceToHost, stream));
                HIP_OK(hipStreamSynchronize(stream));
                for (int64_t k = 0; k < nc; ++k) rp[(size_t)k + 1] = rp[(size_t)k] + (int64_t)hc[(size_t)k];
                nnz = rp[(size_t)nc];
                CHECK(dalloc(arena, &core_col, (size_t)std::max<int64_t>(nnz, 1)));
                CHECK(dalloc(arena, &core_val, (size_t)std::max<int64_t>(nnz, 1)));
                HIP_OK(hipMemcpyAsync(core_rowp, rp.data(), sizeof(int64_t) * (nc + 1), hipMemcpyHostToDevice,
                                      stream));
                rowp_h = core_rowp;
            }
            for (int c = 0; c < 5 && nc >= 2; ++c) {
                const int64_t M = removals(c);
                if (M == 0) continue;
                const int64_t E = nc * M;
                const int nparts = (int)((E + per - 1) / per);
                for (int part = 0; part < nparts; ++part) {
                    const int64_t pe = (E + nparts - 1) / nparts;
                    const int64_t ps = (int64_t)next_pow2((uint64_t)(4 * pe + 64));
                    RkPass P{c, na, nb, part, nparts, nc, M, (uint64_t)ps - 1};
                    HIP_OK(hipMemsetAsync(th, 0xFF, sizeof(uint64_t) * ps, stream));
                    HIP_OK(hipMemsetAsync(tc, 0, sizeof(uint32_t) * ps, stream));
                    HIP_OK(hipMemsetAsync(totals, 0, sizeof(unsigned long long) * 2, stream));
                    const unsigned ge = (unsigned)std::min<int64_t>((E + 255) / 256, 65536);
                    const unsigned gs = (unsigned)std::min<int64_t>((ps + 255) / 256, 65536);
                    hipLaunchKernelGGL((k_rk_count<W>), dim3(ge), dim3(256), 0, stream, core_keys, P, th, tc, err);
                    hipLaunchKernelGGL(k_rk_groups, dim3(gs), dim3(256), 0, stream, (const uint32_t*)tc, (uint64_t)ps,
                                       tg, gstart, gsize, gcap, totals, err);
                    unsigned long long ht[2];
                    unsigned herr = 0;
                    HIP_OK(hipMemcpyAsync(ht, totals, sizeof(ht), hipMemcpyDeviceToHost, stream));
                    HIP_OK(hipMemcpyAsync(&herr, err, sizeof(unsigned), hipMemcpyDeviceToHost, stream));
                    HIP_OK(hipStreamSynchronize(stream));
                    if (herr || (int64_t)ht[0] > gcap || (int64_t)ht[1] > gmcap)
                        return fail(FCIQMC_EOVERFLOW, "H^D construction: %llu groups of %llu entries exceed the "
                                    "pass capacity (%lld, %lld) or its table (flags %u)", ht[0], ht[1],
                                    (long long)gcap, (long long)gmcap, herr);
                    if (ht[0] == 0) continue;
                    HIP_OK(hipMemsetAsync(gfill, 0, sizeof(uint32_t) * ht[0], stream));
                    hipLaunchKernelGGL((k_rk_scatter<W>), dim3(ge), dim3(256), 0, stream, core_keys, P,
                                       (const uint64_t*)th, (const int32_t*)tg, (const int64_t*)gstart, gfill, gm,
                                       gmcap);
                    const unsigned gp = (unsigned)std::min<unsigned long long>((ht[0] + 3) / 4, 65536);
                    hipLaunchKernelGGL((k_rk_pairs<W>), dim3(gp), dim3(256), 0, stream, v, core_keys, P,
                                       (const int64_t*)gstart, (const uint32_t*)gsize, (int64_t)ht[0],
                                       (const uint64_t*)gm, cnt, (const int64_t*)rowp_h, rfill, core_col, core_val);
                    HIP_OK(hipGetLastError());
                }
            }
        }
        HIP_OK(hipStreamSynchronize(stream));
        unsigned herr = 0;
        HIP_OK(hipMemcpy(&herr, err, sizeof(unsigned), hipMemcpyDeviceToHost));
        if (herr) return fail(FCIQMC_EDEVICE, "H^D construction: table overflow (flags %u)", herr);
        return 0;
    }
    int set_collect(bool on) override {
        if (on == keep_rej) return 0;
        CHECK(discard_pending());
        if (!on) {
            arena.release(rej); arena.release(rej_off); arena.release(rej_cnt);
            rej = nullptr; rej_off = nullptr; rej_cnt = nullptr;
            keep_rej = false;
            cap_rej = 0;
            return 0;
        }
        keep_rej = true;
        cap_rej = std::max<long long>(cap, 1);
        CHECK(dalloc(arena, &rej, (size_t)cap_rej));
        return alloc_rej_index();
    }
    int set_reference(uint64_t a, uint64_t b) override {
        CHECK(discard_pending());  // a queued spawn applied the old reference's initiator rule
        rs.ref_a = a;
        rs.ref_b = b;
        return 0;
    }
    int most_populated(uint64_t& a, uint64_t& b, double& v) override {
        CHECK(refuse_if_broken());
        const int G = std::min(B, 1024);
        Arena tmp;
        double* bv = nullptr;
        uint64_t* bk = nullptr;
        CHECK(dalloc(tmp, &bv, (size_t)G));
        CHECK(dalloc(tmp, &bk, (size_t)2 * G));
        hipLaunchKernelGGL((k_most_populated<W, V>), dim3(G), dim3(kThreads), 0, stream, st[cur], R, B, bv, bk);
        HIP_OK(hipGetLastError());
        std::vector<double> hv((size_t)G);
        std::vector<uint64_t> hk((size_t)2 * G);
        HIP_OK(hipMemcpyAsync(hv.data(), bv, sizeof(double) * G, hipMemcpyDeviceToHost, stream));
        HIP_OK(hipMemcpyAsync(hk.data(), bk, sizeof(uint64_t) * 2 * G, hipMemcpyDeviceToHost, stream));
        HIP_OK(hipStreamSynchronize(stream));
        v = -1.0;
        a = b = ~0ULL;
        for (int g = 0; g < G; ++g) {
            const double x = hv[(size_t)g];
            const uint64_t xa = hk[(size_t)(2 * g)], xb = hk[(size_t)(2 * g + 1)];
            if (x > v || (x == v && (xa < a || (xa == a && xb < b)))) { v = x; a = xa; b = xb; }
        }
        return 0;
    }
    int set_rdm(bool on) override {
        CHECK(discard_pending());  // a queued spawn would not log its draws
        rdm_on = on;
        rdm_n = 0;
        if (!on) {
            arena.release(rdm);
            rdm = nullptr;
            cap_rdm = 0;
        }
        return 0;
    }
    // Room for one RDM record per attempt slot of the next spawn launch.
    int ensure_rdm() {
        if (!rdm_on) return 0;
        const int64_t need = std::max<int64_t>(chunk_next, 1) * kChunk;
        if (need > cap_rdm) {
            const int64_t c = need + need / 4;
            CHECK(regrow(rdm, (size_t)c));
            cap_rdm = c;
        }
        return 0;
    }
    const void* rdm_records() const override { return rdm; }
    int64_t rdm_count() const override { return rdm_n; }
    void* rej_records() const override { return rej; }
    int64_t* rej_offsets() const override { return rej_off; }
    int32_t* rej_counts() const override { return rej_cnt; }
    const void* current_store() const override { return &st[cur]; }
    const void* previous_store() const override { return &st[1 - cur]; }
    int bucket_entries() const override { return R; }
    int64_t core_size() const override { return ncore; }
    int64_t core_nnz() const override { return nnz; }
    const std::vector<uint64_t>& core_dets() const override { return core_host; }
    int core_row(int64_t k, int32_t* cols, double* vals, int64_t cap, int64_t* n_out) override {
        if (k < 0 || k >= ncore)
            return fail(FCIQMC_EINVAL, "row %lld out of range [0, %lld)", (long long)k, (long long)ncore);
        int64_t r[2];
        HIP_OK(hipMemcpy(r, core_rowp + k, sizeof(r), hipMemcpyDeviceToHost));
        const int64_t n = r[1] - r[0], m = std::min(n, std::max<int64_t>(cap, 0));
        if (n_out) *n_out = n;
        if (cols && m > 0) HIP_OK(hipMemcpy(cols, core_col + r[0], sizeof(int32_t) * m, hipMemcpyDeviceToHost));
        if (vals && m > 0) HIP_OK(hipMemcpy(vals, core_val + r[0], sizeof(double) * m, hipMemcpyDeviceToHost));
        return 0;
    }

    int get_walkers(std::vector<uint64_t>& ab, std::vector<double>& vals) override {
        CHECK(refuse_if_broken());
        const Store<V>& s = st[cur];
        int64_t* off = nullptr;
        uint64_t* keys = nullptr;
        double* dv = nullptr;
        Arena tmp;
        CHECK(dalloc(tmp, &off, (size_t)B + 1));
        hipLaunchKernelGGL(k_count_offsets, dim3(1), dim3(1024), 0, stream, s.count, B, off);
        int64_t n = 0;
        HIP_OK(hipMemcpyAsync(&n, off + B, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
        HIP_OK(hipStreamSynchronize(stream));
        CHECK(dalloc(tmp, &keys, (size_t)std::max<int64_t>(n, 1) * W));
        CHECK(dalloc(tmp, &dv, (size_t)std::max<int64_t>(n, 1)));
        hipLaunchKernelGGL((k_extract<W, V>), dim3(std::min(B, 4096)), dim3(kThreads), 0, stream, s, R, off,
                           keys, dv, B);
        HIP_OK(hipGetLastError());
        std::vector<uint64_t> hk((size_t)n * W);
        vals.resize((size_t)n);
        if (n > 0) {
            HIP_OK(hipMemcpyAsync(hk.data(), keys, sizeof(uint64_t) * W * n, hipMemcpyDeviceToHost, stream));
            HIP_OK(hipMemcpyAsync(vals.data(), dv, sizeof(double) * n, hipMemcpyDeviceToHost, stream));
        }
        HIP_OK(hipStreamSynchronize(stream));
        tmp.clear();
        ab.resize((size_t)n * 2);
        for (int64_t i = 0; i < n; ++i) {
            if constexpr (W == 1) { ab[2 * i] = hk[i] & 0xFFFFFFFFULL; ab[2 * i + 1] = hk[i] >> 32; }
            else { ab[2 * i] = hk[2 * i]; ab[2 * i + 1] = hk[2 * i + 1]; }
        }
        return 0;
    }

    // The step's extensions (deterministic space, discarded-spawn records,
    // adaptive shift) run in their own kernel instantiations, so the plain
    // step keeps the code it had without them.
    bool ext() const { return ncore > 0 || keep_rej || rs.adaptive || rdm_on; }
    template <int GEN> void launch_spawn_g(const Store<V>& in, const StepScalars& sc, unsigned blocks) {
        const SysView v = sys->view();
        // the Cauchy-Schwarz generators keep J and SK in LDS
        const size_t lds = (GEN >= 3 && v.N <= kCsLdsMaxN) ? 2 * sizeof(double) * (size_t)v.N * (size_t)v.N : 0;
        if (ext())
            hipLaunchKernelGGL((k_spawn<W, V, GEN, true>), dim3(blocks), dim3(kThreads), lds, stream, v, in, sc,
                               rec2, scur, ctl, cmap, cap_cmap);
        else
            hipLaunchKernelGGL((k_spawn<W, V, GEN, false>), dim3(blocks), dim3(kThreads), lds, stream, v, in, sc,
                               rec2, scur, ctl, cmap, cap_cmap);
    }
    // Spawn from store `in` with `grid` workgroups (the kernel reads the
    // chunk count from the device and strides over it).
    int launch_spawn(const Store<V>& in, const StepScalars& sc, int64_t grid) {
        const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(grid, 1 << 30));
        switch (rs.gen) {
            case FCIQMC_GEN_UNIFORM: launch_spawn_g<0>(in, sc, blocks); break;
            case FCIQMC_GEN_LATTICE: launch_spawn_g<1>(in, sc, blocks); break;
            case FCIQMC_GEN_PCHB: launch_spawn_g<2>(in, sc, blocks); break;
            case FCIQMC_GEN_CS: launch_spawn_g<3>(in, sc, blocks); break;
            default: launch_spawn_g<4>(in, sc, blocks); break;
        }
        HIP_OK(hipGetLastError());
        return 0;
    }

    // Outcome of a launched step whose scalars are in hctl: done, or the
    // capacities fixed for a replay of the same step, or an error.
    int settle(int64_t t, int& retries, bool& done) {
        const unsigned flags = hctl->flags;
        done = flags == 0;
        if (done) return 0;
        dirty = true;
        if (flags & kFlagBloom)
            return fail(FCIQMC_EOVERFLOW, "a spawn exceeded 2^30 walkers at step %lld (time step too large)",
                        (long long)t);
        if (flags & kFlagPop)
            return fail(FCIQMC_EOVERFLOW, "a walker number exceeded the int32 range at step %lld", (long long)t);
        if (flags & kFlagSpin) return fail(FCIQMC_EDEVICE, "LDS hash claim did not complete");
        ++retries;
        if (retries > 24) return fail(FCIQMC_EOVERFLOW, "step %lld did not fit after 24 capacity growths", (long long)t);
        if (flags & (kFlagTable | kFlagStore)) {
            CHECK(grow_buckets());
            dirty = false;
            return 0;
        }
        if (flags & kFlagSpawnCap) {
            CHECK(recover());
            dirty = false;
            return 0;
        }
        return fail(FCIQMC_EDEVICE, "device flags 0x%x", flags);
    }

    // Accept the step: swap the stores, take the next step's sizes; double
    // the bucket count when the mean occupancy has grown past the bound.
    int complete(Ctl& out) {
        cur = 1 - cur;
        ada_clean = true;
        att_next = hctl->attempts;
        rec_need = hctl->rec_need;
        out = *hctl;
        out.nref = hctl->nref_out;
        const bool grow = hctl->ndets > kMaxMeanOccupancy * (int64_t)B && (int64_t)B * 2 <= max_b && !fixed_b;
        if (!grow && hctl->chunks <= cap_cmap && rec_need <= cap) {
            chunk_next = hctl->chunks;
            return 0;
        }
        CHECK(discard_pending());  // a queued spawn used buffers that change now
        if (grow) return grow_buckets();
        CHECK(ensure_cmap());
        return ensure_slabs(rec_need);
    }

    // Launch the step alone until it fits.  With `ahead`, the next step's
    // spawn is queued behind this step's post work while the host waits for
    // the scalars.
    int run_alone(int64_t t, double S, int& retries, bool ahead) {
        for (;;) {
            CHECK(ensure_rej());
            CHECK(ensure_rdm());
            const StepScalars sc = scalars(t, S, 0);
            const int set = sampled(t) ? (int)(t & 1) : -1;
            if (!pending) {
                mark(set, 0);
                rdm_n = rdm_on ? chunk_next * kChunk : 0;
                CHECK(launch_spawn(st[cur], sc, chunk_next));
                mark(set, 1);
            }
            pending = false;
            CHECK(launch_merge_post(sc, set));
            if (ahead) {
                const int nset = sampled(t + 1) ? (int)((t + 1) & 1) : -1;
                mark(nset, 0);
                CHECK(launch_spawn(st[1 - cur], scalars(t + 1, S, 0), chunk_next + chunk_next / 8 + 64));
                mark(nset, 1);
                HIP_OK(hipGetLastError());
                pending = true;
                pending_t = t + 1;
            }
            HIP_OK(hipEventSynchronize(ev_copy));
            if (hctl->flags && pending) {
                // the queued spawn ran on a failed step's output: let it end;
                // its record counts only enlarge the recovered slabs
                HIP_OK(hipStreamSynchronize(stream));
                pending = false;
            }
            bool done = false;
            CHECK(settle(t, retries, done));
            if (done) return collect(set);
        }
    }

    int step_once(int64_t t, double S, Ctl& out, int& retries, int64_t& attempts) override {
        CHECK(refuse_if_broken());
        retries = 0;
        attempts = att_next;
        if (pending && pending_t != t) CHECK(discard_pending());
        if (dirty) {
            CHECK(recover());
            dirty = false;
        }
        // with RDM logging the next spawn is not queued ahead: it would
        // overwrite this step's records before the pair has read them
        CHECK(run_alone(t, S, retries, !rdm_on));
        return complete(out);
    }

    // Batched stepping: the instance descriptor of step t and its spawn chunks.
    int batch_prepare(int64_t t, double S, Inst<W, V>& d, int64_t& chunks) {
        CHECK(refuse_if_broken());
        CHECK(discard_pending());
        if (dirty) {
            CHECK(recover());
            dirty = false;
        }
        d.sys = sys->view();
        d.in = st[cur];
        d.out = st[1 - cur];
        d.sc = scalars(t, S, 0);
        d.rec2 = rec2; d.soff = soff; d.scur = scur; d.rel = rel; d.need_b = need_b; d.recs_b = recs_b;
        d.nw_b = nw_b; d.en_b = en_b; d.fpos = fpos; d.fcnt = fcnt; d.ctl = ctl;
        d.cmap = cmap; d.cmap_cap = cap_cmap;
        chunks = chunk_next;
        return 0;
    }
    // The batch's read-back of this instance; a flagged step is replayed alone.
    int batch_finish(int64_t t, double S, const Ctl& c, Ctl& out, int& retries, int64_t& attempts) {
        retries = 0;
        attempts = att_next;
        *hctl = c;
        bool done = false;
        CHECK(settle(t, retries, done));
        if (!done) CHECK(run_alone(t, S, retries, false));
        return complete(out);
    }
    void set_stream(hipStream_t s) override { stream = s; }
    hipStream_t get_stream() const override { return stream; }
    int kind() const override { return kind_of<W, V>(); }
    int64_t ndets() const override { return hctl ? hctl->ndets : 0; }
    int rebucket(int buckets) override {
        if (buckets == B) return 0;
        CHECK(refuse_if_broken());
        std::vector<uint64_t> ab;
        std::vector<double> vals;
        CHECK(get_walkers(ab, vals));
        broken = true;  // until the population is back in the new store
        free_buckets();
        B = buckets;
        CHECK(alloc_buckets());
        cur = 0;
        dirty = false;
        return import(ab.data(), vals.data(), (int64_t)vals.size());
    }
};

struct fciqmc_run {
    fciqmc_system* sys = nullptr;
    fciqmc_params p{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::unique_ptr<EngineBase> eng;
    double h00 = 0.0;
    uint64_t ref_a = 0, ref_b = 0;
    // reference of the projected energy (re-chosen if asked) and
    // H_PP - H_00 of it
    uint64_t proj_a = 0, proj_b = 0;
    double hproj = 0.0;
    int64_t t = 0;
    double S = 0.0;
    int vary = 0;
    int64_t t_last = 0;
    double nw_last = 0.0;
    int64_t t_vary = -1;
    int64_t t_set = 0;              // step at which the population was last set
    double xi = 0.0;                // restoring strength of the shift update
    std::vector<double> nw_ring;    // N_w(t) of the last A+1 steps, indexed t mod (A+1)
    std::vector<fciqmc_step_stats> hist;
    fciqmc_batch* batch = nullptr;  // set while the run steps inside a batch
    int batch_slot = -1;            // its position among the batch's members
    fciqmc_pair* pair = nullptr;    // set while the run is one replica of a pair
    bool rechoose_pending = false;  // the reference is re-chosen before the next step
    ~fciqmc_run() {
        eng.reset();
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

// Population control (Sec. I leaves the update open).  Reading: S stays 0
// (relative to H_00) until N_w first reaches the target N_t.  At that step T
// the shift is set from the measured growth rate,
// S = -ln(N_w(T)/N_w(T-L))/(L dtau), L = min(A, steps since the population was
// set).  From then on, every A steps,
//   S <- S - zeta/(A dtau) ln(N_w(t)/N_w(t-A)) - xi/(A dtau) ln(N_w(t)/N_t),
// the damped control of the original method plus the restoring term of
// Yang, Pahl and Brand (J. Chem. Phys. 153, 174103 (2020)); xi = zeta^2/4 by
// default.  An extinct population (N_w = 0) leaves S unchanged.
static void shift_update(fciqmc_run* r, double nw) {
    const int64_t T = r->t;
    const int64_t A = (int64_t)r->p.shift_interval;
    if (!r->vary) {
        if (nw >= r->p.walker_target) {
            r->vary = 1;
            int64_t L = std::min<int64_t>(T - r->t_set, A);
            if (L > 0) {
                const double nw_prev = r->nw_ring[(size_t)((T - L) % (A + 1))];
                const double c = 1.0 / ((double)L * r->p.tau);
                const double ratio = nw / nw_prev;
                const double l = std::log(ratio);
                const double dS = c * l;
                r->S = 0.0 - dS;
            }
            r->t_last = T;
            r->nw_last = nw;
            r->t_vary = T;
        }
    } else if (T - r->t_last == A && nw > 0.0) {
        const double at = (double)r->p.shift_interval * r->p.tau;
        const double c1 = r->p.shift_damping / at;
        const double c2 = r->xi / at;
        const double l1 = std::log(nw / r->nw_last);
        const double l2 = std::log(nw / r->p.walker_target);
        const double d1 = c1 * l1;
        const double d2 = c2 * l2;
        const double s1 = r->S - d1;
        r->S = s1 - d2;
        r->t_last = T;
        r->nw_last = nw;
    }
    r->nw_ring[(size_t)(T % (A + 1))] = nw;
}


// Advance the run's clock by the completed step: shift update and the
// recorded per-step estimators.
static int device_diag(const fciqmc_system* sys, hipStream_t stream, uint64_t a, uint64_t b, double* out);

// Reference of the projected energy (Sec. IV).  Reading: with re-choice on,
// once the population has relaxed for ceil(1/dtau) steps after the shift
// started varying, the most populated determinant takes over for the
// following steps (ties: ascending alpha, then beta); H_00 stays the energy
// zero.
static int rechoose_reference(fciqmc_run* run) {
    uint64_t a = 0, b = 0;
    double v = 0.0;
    CHECK(run->eng->most_populated(a, b, v));
    if (v <= 0.0 || (a == run->proj_a && b == run->proj_b)) return 0;
    double hpp = 0.0;
    CHECK(device_diag(run->sys, run->eng->get_stream(), a, b, &hpp));
    CHECK(run->eng->set_reference(a, b));
    run->proj_a = a;
    run->proj_b = b;
    run->hproj = hpp - run->h00;
    return 0;
}

static int64_t rechoose_step(const fciqmc_run* run) {
    return run->t_vary + (int64_t)std::ceil(1.0 / run->p.tau);
}

static void record_step(fciqmc_run* run, const Ctl& c, int retries, int64_t attempts, fciqmc_step_stats* out) {
    run->t += 1;
    shift_update(run, c.nw);
    fciqmc_step_stats s{};
    s.iter = run->t;
    s.nw = c.nw;
    s.nref = c.nref;
    s.enum_ = c.enum_;
    s.shift = run->S;
    const double eref = run->h00 + run->sys->e_core;
    const double q = c.enum_ / c.nref;
    s.e_proj = (eref + run->hproj) + q;
    s.ndets = c.ndets;
    s.attempts = attempts;
    s.spawns = c.nrec_out;
    s.vary_shift = run->vary;
    s.retries = retries;
    run->hist.push_back(s);
    if (out) *out = s;
    if (run->p.ref_rechoose && run->t_vary >= 0 && run->t == rechoose_step(run)) run->rechoose_pending = true;
}

// ---------------------------------------------------------------------------
// Batches: runs that advance together, one set of launches per step for all
// of them.  Runs are grouped by engine kind (determinant width and value
// type); each group launches one spawn kernel per excitation generator, one
// annihilation kernel and one post kernel, and all groups share one
// read-back and one synchronisation per step.
// ---------------------------------------------------------------------------
struct BatchGroupBase {
    std::vector<fciqmc_run*> runs;  // ordered by excitation generator
    virtual ~BatchGroupBase() {}
    virtual int prepare(hipStream_t s) = 0;
    // the whole step in one cooperative launch (after prepare)
    virtual int launch_persistent(hipStream_t s) = 0;
    virtual int launch_spawn(hipStream_t s, int grid) = 0;
    virtual int launch_annihilate(hipStream_t s, int grid) = 0;
    virtual int launch_post(hipStream_t s) = 0;
    // after the stream synchronised: accept or replay each run's step
    virtual int finish(fciqmc_step_stats* row) = 0;
};

template <int W, class V> struct BatchGroup : BatchGroupBase {
    using E = Engine<W, V>;
    Arena arena;
    size_t cap = 0;             // instances the buffers hold
    char* hbuf = nullptr;       // pinned: Inst[cap], bucket prefix [cap+1], chunk prefixes [cap+kGens],
                                // diagonal work-item prefix [cap+1]
    char* dbuf = nullptr;       // device copy of hbuf
    Ctl* hctl = nullptr;        // pinned, written by the post kernel, one per instance
    int g0[kGens + 1] = {};     // first instance of each generator, g0[kGens] = n
    int64_t ctot[kGens] = {};
    int64_t btot = 0;
    int64_t ftot = 0;           // work items of the new-diagonal kernel
    size_t flds = 0;            // its LDS bytes (largest molecular member)
    size_t flds_tab = 0;        // the same without the orbital lists (persistent launch)

    Arena arena_bar;            // holds bar (kept across reserve())
    ~BatchGroup() override {
        if (hbuf) (void)hipHostFree(hbuf);
        if (hctl) (void)hipHostFree(hctl);
        arena.clear();
        arena_bar.clear();
    }
    E* eng(size_t i) const { return static_cast<E*>(runs[i]->eng.get()); }
    GridBar* bar = nullptr;     // grid barrier of the persistent launch
    bool bar_dirty = true;      // reset it before the next persistent launch
    int max_blocks[kGens + 1] = {};  // co-resident workgroups per kernel variant (0 = not yet known)
    size_t mb_lds[kGens + 1] = {};   // the dynamic LDS size they were found for
    static size_t bytes_for(size_t n) { return sizeof(Inst<W, V>) * n + sizeof(int64_t) * (4 * n + kGens + 3); }
    int64_t* bfirst(char* base) const { return reinterpret_cast<int64_t*>(base + sizeof(Inst<W, V>) * cap); }
    int64_t* cfirst(char* base) const { return bfirst(base) + cap + 1; }
    int64_t* ffirst(char* base) const { return cfirst(base) + cap + kGens; }
    int64_t* pfirst(char* base) const { return ffirst(base) + cap + 1; }  // chunks over all members

    int reserve(size_t n) {
        if (n <= cap) return 0;
        const size_t c = std::max<size_t>({n, 2 * cap, 8});
        if (hbuf) (void)hipHostFree(hbuf);
        if (hctl) (void)hipHostFree(hctl);
        hbuf = nullptr;
        hctl = nullptr;
        arena.clear();
        cap = 0;
        HIP_OK(hipHostMalloc((void**)&hbuf, bytes_for(c), hipHostMallocDefault));
        HIP_OK(hipHostMalloc((void**)&hctl, sizeof(Ctl) * c, hipHostMallocCoherent));  // written by kernels
        CHECK(dalloc(arena, &dbuf, bytes_for(c)));
        cap = c;
        return 0;
    }

    int prepare(hipStream_t s) override {
        const size_t n = runs.size();
        if (n == 0) return 0;
        CHECK(reserve(n));
        Inst<W, V>* hi = reinterpret_cast<Inst<W, V>*>(hbuf);
        int64_t* bf = bfirst(hbuf);
        int64_t* cf = cfirst(hbuf);
        int64_t* ff = ffirst(hbuf);
        std::vector<int64_t> chunks(n);
        btot = 0;
        ftot = 0;
        flds = 0;
        flds_tab = 0;
        for (size_t i = 0; i < n; ++i) {
            if (runs[i]->rechoose_pending) {
                CHECK(rechoose_reference(runs[i]));
                runs[i]->rechoose_pending = false;
            }
            CHECK(eng(i)->batch_prepare(runs[i]->t, runs[i]->S, hi[i], chunks[i]));
            bf[i] = btot;
            btot += eng(i)->B;
            ff[i] = ftot;
            if (!hi[i].sys.onsite) {
                ftot += fresh_items(eng(i)->B);
                flds = std::max(flds, fresh_lds_bytes(hi[i].sys.N, hi[i].sys.na + hi[i].sys.nb));
                flds_tab = std::max(flds_tab, fresh_lds_bytes(hi[i].sys.N, 0));
            }
        }
        bf[n] = btot;
        ff[n] = ftot;
        {
            int64_t* pf = pfirst(hbuf);
            int64_t c = 0;
            for (size_t i = 0; i < n; ++i) {
                pf[i] = c;
                c += chunks[i];
                hi[i].gen = runs[i]->p.excitgen;
            }
            pf[n] = c;
        }
        // generator ranges; range g keeps its chunk prefix in cf[g0[g] + g .. g0[g+1] + g]
        int k = 0;
        for (int g = 0; g < kGens; ++g) {
            g0[g] = k;
            while (k < (int)n && runs[k]->p.excitgen == g) ++k;
        }
        g0[kGens] = (int)n;
        for (int g = 0; g < kGens; ++g) {
            int64_t c = 0;
            for (int i = g0[g]; i < g0[g + 1]; ++i) {
                cf[i + g] = c;
                c += chunks[i];
            }
            cf[g0[g + 1] + g] = c;
            ctot[g] = c;
        }
        HIP_OK(hipMemcpyAsync(dbuf, hbuf, bytes_for(cap), hipMemcpyHostToDevice, s));
        return 0;
    }
    // One launch for the whole step of every member: a kernel variant with
    // the generator fixed when all members share one of the table-free
    // generators, else with the generator chosen per member; as many
    // workgroups as can be resident together (at most the largest phase's
    // work items); members' step scalars poisoned beforehand so that a
    // launch whose barrier failed leaves them flagged.
    int launch_persistent(hipStream_t s) override {
        if (runs.empty()) return 0;
        if (!bar) {
            CHECK(dalloc(arena_bar, &bar, 1));
            bar_dirty = true;
        }
        if (bar_dirty) {
            HIP_OK(hipMemsetAsync(bar, 0, sizeof(GridBar), s));
            bar_dirty = false;
        }
        int gen = runs[0]->p.excitgen;
        for (auto* r : runs)
            if (r->p.excitgen != gen) gen = -1;
        if (gen > 2) gen = -1;
        const void* fn;
        switch (gen) {
            case 0: fn = reinterpret_cast<const void*>(&k_batch_step<W, V, 0>); break;
            case 1: fn = reinterpret_cast<const void*>(&k_batch_step<W, V, 1>); break;
            case 2: fn = reinterpret_cast<const void*>(&k_batch_step<W, V, 2>); break;
            default: fn = reinterpret_cast<const void*>(&k_batch_step<W, V, -1>); break;
        }
        // dynamic LDS: the new-diagonal tables of the largest molecular member
        const size_t lds = std::max<size_t>(flds_tab, sizeof(double));
        int& mb = max_blocks[gen + 1];
        if (mb == 0 || mb_lds[gen + 1] != lds) {
            int per_cu = 0, cus = 0, dev = 0;
            HIP_OK(hipGetDevice(&dev));
            HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThreads, lds));
            mb = std::max(1, per_cu) * std::max(1, cus);
            mb_lds[gen + 1] = lds;
        }
        const int64_t work = std::max<int64_t>({pfirst(hbuf)[runs.size()], btot, ftot, (int64_t)runs.size(), 1});
        const unsigned grid = (unsigned)std::min<int64_t>(work, mb);
        for (size_t i = 0; i < runs.size(); ++i) hctl[i].flags = kFlagSpin;
        const Inst<W, V>* di = reinterpret_cast<const Inst<W, V>*>(dbuf);
        const int64_t* cf = pfirst(dbuf);
        const int64_t* bf = bfirst(dbuf);
        const int64_t* ff = ffirst(dbuf);
        int k = (int)runs.size();
        GridBar* gb = bar;
        Ctl* ho = hctl;
        void* args[] = {&di, &cf, &bf, &ff, &k, &gb, &ho};
        HIP_OK(hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kThreads), args, lds, s));
        return 0;
    }
    int launch_spawn(hipStream_t s, int grid) override {
        if (runs.empty()) return 0;
        const Inst<W, V>* di = reinterpret_cast<const Inst<W, V>*>(dbuf);
        const int64_t* cf = cfirst(dbuf);
        for (int g = 0; g < kGens; ++g) {
            if (ctot[g] == 0) continue;
            const unsigned gs = (unsigned)(grid > 0 ? std::min<int64_t>(ctot[g], grid) : ctot[g]);
            const int k = g0[g + 1] - g0[g];
            const Inst<W, V>* ig = di + g0[g];
            const int64_t* fg = cf + g0[g] + g;
            if (g == FCIQMC_GEN_UNIFORM)
                hipLaunchKernelGGL((k_spawn_batch<W, V, 0>), dim3(gs), dim3(kThreads), 0, s, ig, fg, k);
            else if (g == FCIQMC_GEN_LATTICE)
                hipLaunchKernelGGL((k_spawn_batch<W, V, 1>), dim3(gs), dim3(kThreads), 0, s, ig, fg, k);
            else if (g == FCIQMC_GEN_PCHB)
                hipLaunchKernelGGL((k_spawn_batch<W, V, 2>), dim3(gs), dim3(kThreads), 0, s, ig, fg, k);
            else if (g == FCIQMC_GEN_CS)
                hipLaunchKernelGGL((k_spawn_batch<W, V, 3>), dim3(gs), dim3(kThreads), 0, s, ig, fg, k);
            else
                hipLaunchKernelGGL((k_spawn_batch<W, V, 4>), dim3(gs), dim3(kThreads), 0, s, ig, fg, k);
        }
        HIP_OK(hipGetLastError());
        return 0;
    }
    int launch_annihilate(hipStream_t s, int grid) override {
        if (runs.empty()) return 0;
        const unsigned gs = (unsigned)(grid > 0 ? std::min<int64_t>(btot, grid) : btot);
        hipLaunchKernelGGL((k_annihilate_batch<W, V>), dim3(gs), dim3(kThreads), 0, s,
                           reinterpret_cast<const Inst<W, V>*>(dbuf), (const int64_t*)bfirst(dbuf), (int)runs.size());
        if (ftot > 0)
            hipLaunchKernelGGL((k_fresh_batch<W, V>), dim3((unsigned)std::min<int64_t>(ftot, 4096)), dim3(kThreads),
                               flds, s, reinterpret_cast<const Inst<W, V>*>(dbuf), (const int64_t*)ffirst(dbuf),
                               (int)runs.size());
        HIP_OK(hipGetLastError());
        return 0;
    }
    int launch_post(hipStream_t s) override {
        if (runs.empty()) return 0;
        hipLaunchKernelGGL((k_post_batch<W, V>), dim3((unsigned)runs.size()), dim3(kPostThreads), 0, s,
                           reinterpret_cast<const Inst<W, V>*>(dbuf), hctl);
        HIP_OK(hipGetLastError());
        return 0;
    }
    int finish(fciqmc_step_stats* row) override {
        int rc = 0;
        std::string msg;
        for (size_t i = 0; i < runs.size(); ++i)
            if (hctl[i].flags & kFlagSpin) bar_dirty = true;
        for (size_t i = 0; i < runs.size(); ++i) {
            fciqmc_run* r = runs[i];
            Ctl out{};
            int retries = 0;
            int64_t attempts = 0;
            const int e = eng(i)->batch_finish(r->t, r->S, hctl[i], out, retries, attempts);
            if (e) {
                if (!rc) {
                    rc = e;
                    msg = "batch member " + std::to_string(r->batch_slot) + ": " + g_err;
                }
                continue;
            }
            record_step(r, out, retries, attempts, row ? row + r->batch_slot : nullptr);
        }
        if (rc) g_err = msg;
        return rc;
    }
};

static std::unique_ptr<BatchGroupBase> make_group(int kind) {
    switch (kind) {
        case kind_of<1, int32_t>(): return std::unique_ptr<BatchGroupBase>(new BatchGroup<1, int32_t>());
        case kind_of<1, double>(): return std::unique_ptr<BatchGroupBase>(new BatchGroup<1, double>());
        case kind_of<2, int32_t>(): return std::unique_ptr<BatchGroupBase>(new BatchGroup<2, int32_t>());
        default: return std::unique_ptr<BatchGroupBase>(new BatchGroup<2, double>());
    }
}

struct fciqmc_batch {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<fciqmc_run*> members;          // in order of addition
    std::unique_ptr<BatchGroupBase> group[4];  // by engine kind
    int grid_spawn = 0, grid_ann = 0;          // workgroups per launch, 0 = one per work item
    int persistent = 0;                        // 1: the step in one cooperative launch per group
    bool profile = false;
    hipEvent_t ev[kKernels + 1]{};
    double kms[kKernels]{};
    int64_t ksteps = 0;
    ~fciqmc_batch() {
        if (stream) (void)hipStreamSynchronize(stream);
        if (profile)
            for (auto& e : ev) (void)hipEventDestroy(e);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

static void batch_detach(fciqmc_batch* b, fciqmc_run* r) {
    (void)hipStreamSynchronize(b->stream);
    auto& g = b->group[r->eng->kind()]->runs;
    g.erase(std::find(g.begin(), g.end(), r));
    b->members.erase(std::find(b->members.begin(), b->members.end(), r));
    for (size_t i = 0; i < b->members.size(); ++i) b->members[i]->batch_slot = (int)i;
    r->eng->set_stream(r->stream);
    r->batch = nullptr;
    r->batch_slot = -1;
}

// One step of every member: all launches queued, one synchronisation, then
// each run accepts its step (or replays it alone after a capacity flag).
static int batch_step_once(fciqmc_batch* b, fciqmc_step_stats* row) {
    for (auto& g : b->group)
        if (g) CHECK(g->prepare(b->stream));
    if (b->profile) HIP_OK(hipEventRecord(b->ev[0], b->stream));
    if (b->persistent) {
        // the whole step in one launch per group: its time is counted as spawn
        for (auto& g : b->group)
            if (g) CHECK(g->launch_persistent(b->stream));
        if (b->profile) {
            HIP_OK(hipEventRecord(b->ev[1], b->stream));
            HIP_OK(hipEventRecord(b->ev[2], b->stream));
            HIP_OK(hipEventRecord(b->ev[3], b->stream));
        }
    } else {
        for (auto& g : b->group)
            if (g) CHECK(g->launch_spawn(b->stream, b->grid_spawn));
        if (b->profile) HIP_OK(hipEventRecord(b->ev[1], b->stream));
        for (auto& g : b->group)
            if (g) CHECK(g->launch_annihilate(b->stream, b->grid_ann));
        if (b->profile) HIP_OK(hipEventRecord(b->ev[2], b->stream));
        for (auto& g : b->group)
            if (g) CHECK(g->launch_post(b->stream));
        if (b->profile) HIP_OK(hipEventRecord(b->ev[3], b->stream));
    }
    HIP_OK(hipStreamSynchronize(b->stream));
    if (b->profile) {
        for (int i = 0; i < kKernels; ++i) {
            float ms = 0.f;
            HIP_OK(hipEventElapsedTime(&ms, b->ev[i], b->ev[i + 1]));
            b->kms[i] += ms;
        }
        ++b->ksteps;
    }
    int rc = 0;
    std::string msg;
    for (auto& g : b->group)
        if (g) {
            const int e = g->finish(row);
            if (e && !rc) {
                rc = e;
                msg = g_err;
            }
        }
    if (rc) g_err = msg;
    return rc;
}

extern "C" {

const char* fciqmc_last_error(void) { return g_err.c_str(); }

void fciqmc_params_default(fciqmc_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->tau = 0.01;
    p->walker_target = 1e4;
    p->n_initial = 10.0;
    p->initiator_na = -1.0;
    p->mode = FCIQMC_MODE_INTEGER;
    p->c_min = 1.0;
    p->excitgen = FCIQMC_GEN_UNIFORM;
    p->p_single = -1.0;
    p->p_opp = -1.0;
    p->seed = 1;
    p->replica_id = 0;
    p->shift_damping = 0.05;
    p->shift_restore = -1.0;
    p->shift_interval = 10;
    p->conv_tol = 1e-3;
    p->equil_steps = -1;
}

int fciqmc_load_integrals(int n_orb, int n_alpha, int n_beta, double e_core, const double* h1,
                          const double* eri_packed, int64_t eri_len, fciqmc_system** out) {
    if (!out || !h1 || !eri_packed) return fail(FCIQMC_EINVAL, "null argument");
    *out = nullptr;
    if (n_orb < 1 || n_orb > 63) return fail(FCIQMC_EINVAL, "n_orb must be in [1, 63] (got %d)", n_orb);
    if (n_alpha < 0 || n_beta < 0 || n_alpha > n_orb || n_beta > n_orb)
        return fail(FCIQMC_EINVAL, "electron counts must lie in [0, n_orb]");
    if (n_alpha + n_beta < 1) return fail(FCIQMC_EINVAL, "no electrons");
    if ((n_alpha == 0 || n_alpha == n_orb) && (n_beta == 0 || n_beta == n_orb))
        return fail(FCIQMC_EINVAL, "the determinant space holds a single determinant");
    const int64_t M = (int64_t)n_orb * (n_orb + 1) / 2;
    if (eri_len != M * (M + 1) / 2)
        return fail(FCIQMC_EINVAL, "eri_len must be M(M+1)/2 = %lld for n_orb = %d", (long long)(M * (M + 1) / 2), n_orb);
    for (int p = 0; p < n_orb; ++p)
        for (int q = 0; q < n_orb; ++q) {
            if (!std::isfinite(h1[p * n_orb + q])) return fail(FCIQMC_EINVAL, "h1 has a non-finite entry");
            if (h1[p * n_orb + q] != h1[q * n_orb + p]) return fail(FCIQMC_EINVAL, "h1 is not symmetric at (%d,%d)", p, q);
        }
    for (int64_t i = 0; i < eri_len; ++i)
        if (!std::isfinite(eri_packed[i])) return fail(FCIQMC_EINVAL, "eri has a non-finite entry");
    std::unique_ptr<fciqmc_system> s(new fciqmc_system());
    s->N = n_orb; s->na = n_alpha; s->nb = n_beta; s->e_core = e_core;
    HIP_OK(hipGetDevice(&s->device));
    // input structure: which two-electron integrals are non-zero
    bool onsite = true;
    for (int64_t P = 0, idx = 0; P < M && onsite; ++P)
        for (int64_t Q = 0; Q <= P; ++Q, ++idx) {
            if (eri_packed[idx] == 0.0) continue;
            // P = p(p+1)/2 + p is a diagonal pair; both pairs must be the same diagonal pair
            int64_t p = 0;
            while ((p + 1) * (p + 2) / 2 <= P) ++p;
            const bool pdiag = (P == p * (p + 1) / 2 + p);
            if (!(P == Q && pdiag)) onsite = false;
        }
    s->onsite = onsite;
    const int N = n_orb;
    CHECK(dalloc(s->arena, &s->h1, (size_t)N * N));
    CHECK(dalloc(s->arena, &s->eri, (size_t)eri_len));
    CHECK(dalloc(s->arena, &s->J, (size_t)N * N));
    CHECK(dalloc(s->arena, &s->K, (size_t)N * N));
    CHECK(dalloc(s->arena, &s->X, (size_t)N * N));
    CHECK(dalloc(s->arena, &s->SK, (size_t)N * N));
    CHECK(dalloc(s->arena, &s->Hd, (size_t)N));
    CHECK(dalloc(s->arena, &s->U, (size_t)N));
    CHECK(dalloc(s->arena, &s->deg, (size_t)N));
    CHECK(dalloc(s->arena, &s->nbr, (size_t)N * N));
    const int np = N * (N - 1) / 2;
    CHECK(dalloc(s->arena, &s->pair_of, (size_t)std::max(np, 1)));
    HIP_OK(hipMemcpy(s->h1, h1, sizeof(double) * N * N, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(s->eri, eri_packed, sizeof(double) * eri_len, hipMemcpyHostToDevice));
    s->h1_host.assign(h1, h1 + (size_t)N * N);
    s->eri_host.assign(eri_packed, eri_packed + eri_len);
    // lattice neighbour lists: the distinct q != p with h_pq != 0, ascending
    std::vector<int> deg(N, 0), nbr((size_t)N * N, 0);
    for (int p = 0; p < N; ++p)
        for (int q = 0; q < N; ++q)
            if (q != p && h1[p * N + q] != 0.0) nbr[(size_t)p * N + deg[p]++] = q;
    HIP_OK(hipMemcpy(s->deg, deg.data(), sizeof(int) * N, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(s->nbr, nbr.data(), sizeof(int) * N * N, hipMemcpyHostToDevice));
    // probabilities of the lattice generator's 32-bit choices: index k of m
    // is taken by the words x in [ceil(k 2^32/m), ceil((k+1) 2^32/m))
    auto word_share = [](uint64_t k, uint64_t m) {
        const uint64_t first = ((k << 32) + m - 1) / m, next = (((k + 1) << 32) + m - 1) / m;
        return (double)(next - first) * 0x1.0p-32;
    };
    const int ne = n_alpha + n_beta;
    std::vector<double> pe((size_t)ne), pz((size_t)N * N, 0.0);
    for (int e = 0; e < ne; ++e) pe[(size_t)e] = word_share((uint64_t)e, (uint64_t)ne);
    for (int z = 1; z < N; ++z)
        for (int d = 0; d < z; ++d) pz[(size_t)z * N + d] = word_share((uint64_t)d, (uint64_t)z);
    CHECK(dalloc(s->arena, &s->lat_pe, (size_t)ne));
    CHECK(dalloc(s->arena, &s->lat_pz, (size_t)N * N));
    HIP_OK(hipMemcpy(s->lat_pe, pe.data(), sizeof(double) * ne, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(s->lat_pz, pz.data(), sizeof(double) * N * N, hipMemcpyHostToDevice));
    std::vector<int> po((size_t)std::max(np, 1), 0);
    for (int A = 0, c = 0; A < N; ++A)
        for (int B = A + 1; B < N; ++B, ++c) po[c] = A * 64 + B;
    HIP_OK(hipMemcpy(s->pair_of, po.data(), sizeof(int) * po.size(), hipMemcpyHostToDevice));
    SysView v = s->view();
    hipLaunchKernelGGL(k_build_jk, dim3((N * N + 255) / 256), dim3(256), 0, 0, v, s->J, s->K, s->X, s->U, s->Hd,
                       s->SK);
    HIP_OK(hipGetLastError());
    HIP_OK(hipDeviceSynchronize());
    *out = s.release();
    return 0;
}

void fciqmc_free_system(fciqmc_system* sys) { delete sys; }

static int device_diag(const fciqmc_system* sys, hipStream_t stream, uint64_t a, uint64_t b, double* out) {
    Arena tmp;
    uint64_t* d = nullptr;
    double* o = nullptr;
    CHECK(dalloc(tmp, &d, 2));
    CHECK(dalloc(tmp, &o, 1));
    uint64_t h[2] = {a, b};
    HIP_OK(hipMemcpyAsync(d, h, sizeof(h), hipMemcpyHostToDevice, stream));
    hipLaunchKernelGGL(k_hij, dim3(1), dim3(64), 0, stream, sys->view(), d, d, 1LL, o);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(out, o, sizeof(double), hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    tmp.clear();
    return 0;
}

static bool valid_det(const fciqmc_system* s, uint64_t a, uint64_t b) {
    const uint64_t full = (s->N >= 64) ? ~0ULL : ((1ULL << s->N) - 1);
    return (a & ~full) == 0 && (b & ~full) == 0 && __builtin_popcountll(a) == s->na &&
           __builtin_popcountll(b) == s->nb;
}

// Initial walker-store buckets and spawn-record capacity of a run: from the
// hints, else from the walker target (both grow on demand).
static void initial_capacity(const fciqmc_params* p, int& B, long long& spawn_cap) {
    const double target = std::max(1.0, p->walker_target);
    int64_t max_dets = p->max_dets > 0 ? p->max_dets : (int64_t)std::min(target, 16777216.0);
    max_dets = std::max<int64_t>(max_dets, 1024);
    // kBucketOccupancy determinants of the capacity hint per bucket (the store
    // holds R = 1024 per bucket; buckets double when one overflows)
    B = p->buckets_log2 > 0 ? (1 << std::min(p->buckets_log2, 22))
                            : (int)next_pow2((uint64_t)((max_dets + kBucketOccupancy - 1) / kBucketOccupancy));
    spawn_cap = p->max_spawns > 0 ? p->max_spawns : (long long)std::min(std::max(65536.0, 1.0 * target), 33554432.0);
}

// Device bytes a run reserves: a walker store of one bucket per 256 walkers
// of the target (a bucket's LDS table holds about that many determinants
// next to their spawn targets), at least one doubling of the initial store;
// spawn slabs for six records per target walker plus the per-sub-slab
// floor; an import staging buffer for three times the target.
static int64_t reserve_bytes(const fciqmc_system* sys, const fciqmc_params* p) {
    int B = 1;
    long long cap = 0;
    initial_capacity(p, B, cap);
    const int W = p->det_words ? p->det_words : (sys->N <= 32 ? 1 : 2);
    const int64_t vb = p->mode == FCIQMC_MODE_INTEGER ? 4 : 8;
    const int64_t rb = ((8 * W + vb + 4) + 7) / 8 * 8;          // one spawn record
    const double target = std::max(1.0, p->walker_target);
    const int64_t Br = std::max<int64_t>(2 * (int64_t)B, (int64_t)next_pow2((uint64_t)std::ceil(target / 256.0)));
    const int64_t entry = 8 * W + vb + 8 + 4;                     // key, value, diagonal, attempt prefix
    const int64_t store = Br * 1024 * entry + Br * (4 + 8 + 8);
    const int64_t per_bucket = Br * (kSub * (4 + 8 + 8) + 8 * 4);
    // a growing population overshoots the target before the shift holds it
    const double recs = std::max<double>((double)cap, 6.0 * target) + 256.0 * (double)Br;
    const int64_t slabs = (int64_t)(1.25 * recs) * rb;
    const int64_t stage = (int64_t)(3.0 * target) * rb;
    return 2 * store + per_bucket + slabs + stage + (1 << 20);
}

int fciqmc_init(const fciqmc_system* csys, const fciqmc_params* p, void* stream, fciqmc_run** out) {
    if (!csys || !p || !out) return fail(FCIQMC_EINVAL, "null argument");
    *out = nullptr;
    fciqmc_system* sys = const_cast<fciqmc_system*>(csys);
    if (!(p->tau > 0.0) || !std::isfinite(p->tau)) return fail(FCIQMC_EINVAL, "tau must be positive");
    if (p->mode != FCIQMC_MODE_INTEGER && p->mode != FCIQMC_MODE_REAL) return fail(FCIQMC_EINVAL, "unknown mode");
    if (p->excitgen < 0 || p->excitgen >= kGens) return fail(FCIQMC_EINVAL, "unknown excitation generator");
    if (p->excitgen == FCIQMC_GEN_LATTICE && !sys->onsite)
        return fail(FCIQMC_EINVAL, "the lattice generator needs on-site-only two-electron integrals");
    if (p->mode == FCIQMC_MODE_REAL && !(p->c_min > 0.0)) return fail(FCIQMC_EINVAL, "c_min must be positive");
    if (p->shift_interval < 1) return fail(FCIQMC_EINVAL, "shift_interval must be >= 1");
    if (!(p->n_initial > 0.0)) return fail(FCIQMC_EINVAL, "n_initial must be positive");
    if (p->mode == FCIQMC_MODE_INTEGER && (p->n_initial != std::floor(p->n_initial) || p->n_initial > 2e9))
        return fail(FCIQMC_EINVAL, "integer mode needs an integral n_initial below 2e9");
    const int N = sys->N;
    int W = p->det_words;
    if (W == 0) W = N <= 32 ? 1 : 2;
    if (W != 1 && W != 2) return fail(FCIQMC_EINVAL, "det_words must be 0, 1 or 2");
    if (W == 1 && N > 32) return fail(FCIQMC_EINVAL, "one-word determinants need n_orb <= 32");
    std::unique_ptr<fciqmc_run> r(new fciqmc_run());
    r->sys = sys;
    r->p = *p;
    if (stream) r->stream = (hipStream_t)stream;
    else { HIP_OK(hipStreamCreateWithFlags(&r->stream, hipStreamNonBlocking)); r->own_stream = true; }
    uint64_t ra = p->ref_alpha, rb = p->ref_beta;
    if (ra == 0 && rb == 0) {
        ra = sys->na >= 64 ? ~0ULL : ((1ULL << sys->na) - 1);
        rb = sys->nb >= 64 ? ~0ULL : ((1ULL << sys->nb) - 1);
    }
    if (!valid_det(sys, ra, rb)) return fail(FCIQMC_EINVAL, "reference determinant is not a valid determinant");
    r->ref_a = ra; r->ref_b = rb;
    r->proj_a = ra; r->proj_b = rb;
    if (p->excitgen == FCIQMC_GEN_PCHB) CHECK(build_pchb(sys, r->stream));
    CHECK(device_diag(sys, r->stream, ra, rb, &r->h00));
    RunScalars rs{};
    rs.tau = p->tau;
    const int n = sys->na + sys->nb;
    if (p->p_single >= 0.0) rs.p_single = p->p_single;
    else {
        // Appendix A.2: p_sing ~ nN/(nN + n^2 N^2)
        const double nN = (double)n * (double)N;
        const double n2N2 = nN * nN;
        rs.p_single = nN / (nN + n2N2);
    }
    if (p->excitgen == FCIQMC_GEN_LATTICE) rs.p_single = 1.0;
    rs.p_double = 1.0 - rs.p_single;
    if (p->p_opp >= 0.0) rs.p_opp = p->p_opp;
    else {
        const int64_t npair = (int64_t)n * (n - 1) / 2;
        rs.p_opp = npair > 0 ? (double)((int64_t)sys->na * sys->nb) / (double)npair : 0.0;
    }
    rs.n_a = p->initiator_na;
    rs.c_min = p->c_min;
    rs.h00 = r->h00;
    rs.seed = p->seed; rs.replica = p->replica_id;
    rs.ref_a = ra; rs.ref_b = rb;
    rs.gen = p->excitgen;
    rs.adaptive = p->adaptive_shift ? 1 : 0;
    int B = 1;
    long long spawn_cap = 0;
    initial_capacity(p, B, spawn_cap);
    if (W == 1 && p->mode == FCIQMC_MODE_INTEGER) r->eng.reset(new Engine<1, int32_t>(sys, r->stream, rs));
    else if (W == 1) r->eng.reset(new Engine<1, double>(sys, r->stream, rs));
    else if (p->mode == FCIQMC_MODE_INTEGER) r->eng.reset(new Engine<2, int32_t>(sys, r->stream, rs));
    else r->eng.reset(new Engine<2, double>(sys, r->stream, rs));
    int rc;
    if (W == 1 && p->mode == FCIQMC_MODE_INTEGER) rc = static_cast<Engine<1, int32_t>*>(r->eng.get())->init(B, spawn_cap, p->hbm_budget_bytes);
    else if (W == 1) rc = static_cast<Engine<1, double>*>(r->eng.get())->init(B, spawn_cap, p->hbm_budget_bytes);
    else if (p->mode == FCIQMC_MODE_INTEGER) rc = static_cast<Engine<2, int32_t>*>(r->eng.get())->init(B, spawn_cap, p->hbm_budget_bytes);
    else rc = static_cast<Engine<2, double>*>(r->eng.get())->init(B, spawn_cap, p->hbm_budget_bytes);
    if (rc) return rc;
    r->eng->fixed_b = p->buckets_log2 > 0;
    uint64_t ab[2] = {ra, rb};
    double v0 = p->n_initial;
    CHECK(r->eng->set_walkers(ab, &v0, 1));
    if (p->shift_restore >= 0.0) r->xi = p->shift_restore;
    else {
        const double z2 = p->shift_damping * p->shift_damping;
        r->xi = z2 / 4.0;
    }
    r->nw_ring.assign((size_t)p->shift_interval + 1, 0.0);
    r->t_set = 0;
    r->nw_ring[0] = r->eng->last_nw();
    *out = r.release();
    return 0;
}

void pair_detach(fciqmc_run* run);

void fciqmc_free_run(fciqmc_run* run) {
    if (!run) return;
    if (run->batch) batch_detach(run->batch, run);
    if (run->pair) pair_detach(run);
    delete run;
}

int fciqmc_batch_create(void* stream, fciqmc_batch** out) {
    if (!out) return fail(FCIQMC_EINVAL, "null argument");
    *out = nullptr;
    std::unique_ptr<fciqmc_batch> b(new fciqmc_batch());
    if (stream) b->stream = (hipStream_t)stream;
    else { HIP_OK(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking)); b->own_stream = true; }
    *out = b.release();
    return 0;
}

int fciqmc_batch_add(fciqmc_batch* b, fciqmc_run* run) {
    if (!b || !run || !run->eng) return fail(FCIQMC_EINVAL, "null argument");
    if (run->batch) return fail(FCIQMC_EINVAL, "the run already belongs to a batch");
    if (run->eng->core_size() > 0)
        return fail(FCIQMC_EINVAL, "a run with a deterministic space is stepped alone");
    if (run->pair) return fail(FCIQMC_EINVAL, "a replica of a pair is stepped by its pair");
    if (run->p.adaptive_shift) return fail(FCIQMC_EINVAL, "a run with the adaptive shift is stepped alone");
    HIP_OK(hipStreamSynchronize(run->stream));
    const int k = run->eng->kind();
    if (!b->group[k]) b->group[k] = make_group(k);
    auto& g = b->group[k]->runs;
    // keep each group ordered by generator (stable within a generator)
    auto pos = std::upper_bound(g.begin(), g.end(), run, [](const fciqmc_run* a, const fciqmc_run* c) {
        return a->p.excitgen < c->p.excitgen;
    });
    g.insert(pos, run);
    run->batch = b;
    run->batch_slot = (int)b->members.size();
    b->members.push_back(run);
    run->eng->set_stream(b->stream);
    return 0;
}

int fciqmc_batch_remove(fciqmc_batch* b, fciqmc_run* run) {
    if (!b || !run) return fail(FCIQMC_EINVAL, "null argument");
    if (run->batch != b) return fail(FCIQMC_EINVAL, "the run is not a member of this batch");
    batch_detach(b, run);
    return 0;
}

int fciqmc_batch_size(const fciqmc_batch* b) { return b ? (int)b->members.size() : 0; }

int fciqmc_batch_step(fciqmc_batch* b, int n_steps, fciqmc_step_stats* stats) {
    if (!b) return fail(FCIQMC_EINVAL, "null argument");
    if (n_steps < 0) return fail(FCIQMC_EINVAL, "n_steps must be >= 0");
    const size_t m = b->members.size();
    if (m == 0) return 0;
    for (int i = 0; i < n_steps; ++i) CHECK(batch_step_once(b, stats ? stats + (size_t)i * m : nullptr));
    return 0;
}

int fciqmc_batch_set_persistent(fciqmc_batch* b, int on) {
    if (!b) return fail(FCIQMC_EINVAL, "null argument");
    b->persistent = on ? 1 : 0;
    return 0;
}

int fciqmc_batch_profile(fciqmc_batch* b, int enable, double* ms, int64_t* steps) {
    if (!b) return fail(FCIQMC_EINVAL, "null argument");
    if (enable && !b->profile) {
        for (auto& e : b->ev) HIP_OK(hipEventCreate(&e));
        b->profile = true;
    }
    if (ms && steps) {
        for (int i = 0; i < kKernels; ++i) ms[i] = b->kms[i];
        *steps = b->ksteps;
    }
    return 0;
}

// Attempts per second of `steps` batch steps under the current launch shape.
static int batch_rate(fciqmc_batch* b, int steps, double& rate) {
    const size_t m = b->members.size();
    std::vector<fciqmc_step_stats> st((size_t)steps * m);
    HIP_OK(hipStreamSynchronize(b->stream));
    const auto t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < steps; ++i) CHECK(batch_step_once(b, st.data() + (size_t)i * m));
    const auto t1 = std::chrono::steady_clock::now();
    double att = 0.0;
    for (const auto& x : st) att += (double)x.attempts;
    const double sec = std::chrono::duration<double>(t1 - t0).count();
    rate = sec > 0.0 ? att / sec : 0.0;
    return 0;
}

// Bucket count giving about `occ` occupied determinants per bucket.
static int buckets_for(int64_t ndets, int occ) {
    const int64_t b = (ndets + occ - 1) / occ;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 1 << 22));
}

int fciqmc_batch_tune(fciqmc_batch* b, int trial_steps, fciqmc_tune_report* out) {
    if (!b) return fail(FCIQMC_EINVAL, "null argument");
    if (trial_steps < 1) return fail(FCIQMC_EINVAL, "trial_steps must be >= 1");
    fciqmc_tune_report rep{};
    if (b->members.empty()) {
        if (out) *out = rep;
        return 0;
    }
    int trials = 0;
    double best = 0.0;
    CHECK(batch_rate(b, trial_steps, best));
    ++trials;
    rep.rate_initial = best;
    // one persistent launch per step, or separate launches per phase
    {
        const int found = b->persistent;
        b->persistent = 1 - found;
        double rate = 0.0;
        CHECK(batch_rate(b, trial_steps, rate));
        ++trials;
        if (rate > best) best = rate;
        else b->persistent = found;
    }
    // walker-store occupancy: rebucket every member, time, keep the best
    const std::vector<int64_t> start_b = [&] {
        std::vector<int64_t> v;
        for (auto* r : b->members) v.push_back(r->eng->buckets());
        return v;
    }();
    std::vector<int64_t> best_b = start_b;
    int best_occ = 0;
    for (int occ : {128, 256, 384}) {
        for (auto* r : b->members) CHECK(r->eng->rebucket(buckets_for(r->eng->ndets(), occ)));
        double rate = 0.0;
        CHECK(batch_rate(b, trial_steps, rate));
        ++trials;
        if (rate > best) {
            best = rate;
            best_occ = occ;
            best_b.clear();
            for (auto* r : b->members) best_b.push_back(r->eng->buckets());
        }
    }
    if (best_occ == 0)
        for (size_t i = 0; i < b->members.size(); ++i) CHECK(b->members[i]->eng->rebucket((int)start_b[i]));
    else
        for (auto* r : b->members) CHECK(r->eng->rebucket(buckets_for(r->eng->ndets(), best_occ)));
    // persistent grids of the two large launches
    int best_gs = b->grid_spawn, best_ga = b->grid_ann;
    for (int gs : {0, 2048, 8192}) {
        if (gs == best_gs) continue;
        b->grid_spawn = gs;
        double rate = 0.0;
        CHECK(batch_rate(b, trial_steps, rate));
        ++trials;
        if (rate > best) { best = rate; best_gs = gs; }
    }
    b->grid_spawn = best_gs;
    for (int ga : {0, 1024, 4096}) {
        if (ga == best_ga) continue;
        b->grid_ann = ga;
        double rate = 0.0;
        CHECK(batch_rate(b, trial_steps, rate));
        ++trials;
        if (rate > best) { best = rate; best_ga = ga; }
    }
    b->grid_ann = best_ga;
    rep.persistent = b->persistent;
    rep.dets_per_bucket = best_occ;
    rep.grid_spawn = best_gs;
    rep.grid_annihilate = best_ga;
    rep.trials = trials;
    rep.steps = (int64_t)trials * trial_steps;
    rep.rate_best = best;
    if (out) *out = rep;
    return 0;
}

void fciqmc_batch_free(fciqmc_batch* b) {
    if (!b) return;
    while (!b->members.empty()) batch_detach(b, b->members.back());
    delete b;
}

int64_t fciqmc_estimate_bytes(const fciqmc_system* sys, const fciqmc_params* p) {
    if (!sys || !p) return fail(FCIQMC_EINVAL, "null argument");
    return reserve_bytes(sys, p);
}

int64_t fciqmc_run_device_bytes(const fciqmc_run* run) { return run && run->eng ? run->eng->bytes() : 0; }

int fciqmc_profile(fciqmc_run* run, int enable, double* ms, int64_t* steps, int64_t* layout) {
    if (!run || !run->eng) return fail(FCIQMC_ESTATE, "run not initialised");
    if (enable) CHECK(run->eng->enable_profile());
    if (ms && steps) run->eng->kernel_times(ms, steps);
    if (layout) {
        layout[0] = run->eng->buckets();
        layout[1] = run->eng->spawn_capacity();
    }
    return 0;
}

int fciqmc_step(fciqmc_run* run, int n_steps, fciqmc_step_stats* stats) {
    if (!run || !run->eng) return fail(FCIQMC_ESTATE, "run not initialised");
    if (run->batch) return fail(FCIQMC_ESTATE, "the run belongs to a batch: step the batch");
    if (n_steps < 0) return fail(FCIQMC_EINVAL, "n_steps must be >= 0");
    for (int i = 0; i < n_steps; ++i) {
        Ctl c{};
        int retries = 0;
        int64_t attempts = 0;
        if (run->rechoose_pending) {
            CHECK(rechoose_reference(run));
            run->rechoose_pending = false;
        }
        CHECK(run->eng->step_once(run->t, run->S, c, retries, attempts));
        record_step(run, c, retries, attempts, stats ? stats + i : nullptr);
    }
    return 0;
}

// Flyvbjerg-Petersen blocking of a mean and of a ratio of means.
namespace {
struct Level { double err, derr; };

double plateau(const std::vector<Level>& lv) {
    const int n = (int)lv.size();
    for (int i = 0; i + 4 <= n; ++i) {
        bool ok = true;
        for (int j = i + 1; j <= i + 3; ++j)
            if (std::fabs(lv[j].err - lv[i].err) > 2.0 * (lv[i].derr + lv[j].derr)) ok = false;
        if (ok) return lv[i].err;
    }
    double m = 0.0;
    for (int i = 0; i < std::max(1, n - 3); ++i) m = std::max(m, lv[i].err);
    return m;
}

void blocking(std::vector<double> x, std::vector<double> y, double& mx, double& ex, double& my,
              double& ratio, double& eratio) {
    const size_t n0 = x.size();
    mx = 0.0; my = 0.0;
    for (size_t i = 0; i < n0; ++i) { mx += x[i]; my += y[i]; }
    mx /= (double)n0; my /= (double)n0;
    ratio = my != 0.0 ? mx / my : NAN;
    std::vector<Level> lx, lr;
    while (x.size() >= 2) {
        // (co)variances about this level's own means (a level drops the odd
        // last element); the ratio's derivatives at the overall means
        const size_t n = x.size();
        double ax = 0.0, ay = 0.0;
        for (size_t i = 0; i < n; ++i) { ax += x[i]; ay += y[i]; }
        ax /= (double)n; ay /= (double)n;
        double vx = 0.0, vy = 0.0, cxy = 0.0;
        for (size_t i = 0; i < n; ++i) {
            vx += (x[i] - ax) * (x[i] - ax);
            vy += (y[i] - ay) * (y[i] - ay);
            cxy += (x[i] - ax) * (y[i] - ay);
        }
        vx /= (double)n; vy /= (double)n; cxy /= (double)n;
        const double e = std::sqrt(vx / (double)(n - 1));
        const double de = e / std::sqrt(2.0 * (double)(n - 1));
        lx.push_back({e, de});
        const double vr = (vx / (my * my) - 2.0 * mx * cxy / (my * my * my) + mx * mx * vy / (my * my * my * my)) /
                          (double)(n - 1);
        const double er = std::sqrt(std::max(vr, 0.0));
        lr.push_back({er, er / std::sqrt(2.0 * (double)(n - 1))});
        const size_t m = n / 2;
        for (size_t i = 0; i < m; ++i) {
            x[i] = 0.5 * (x[2 * i] + x[2 * i + 1]);
            y[i] = 0.5 * (y[2 * i] + y[2 * i + 1]);
        }
        x.resize(m);
        y.resize(m);
    }
    ex = lx.empty() ? NAN : plateau(lx);
    eratio = lr.empty() ? NAN : plateau(lr);
}
}  // namespace

int fciqmc_energy(const fciqmc_run* run, fciqmc_energy_report* out) {
    if (!run || !out) return fail(FCIQMC_EINVAL, "null argument");
    std::memset(out, 0, sizeof(*out));
    const double eref = run->h00 + run->sys->e_core;
    out->e_ref = eref;
    out->steps_done = run->t;
    out->e_proj = out->e_proj_err = out->shift = out->shift_err = NAN;
    if (run->t_vary < 0) return 0;
    const int64_t after = run->t - run->t_vary;
    int64_t equil = run->p.equil_steps;
    if (equil < 0) equil = std::max<int64_t>((int64_t)std::ceil(1.0 / run->p.tau), after / 5);
    int64_t first = run->t_vary + equil;  // first step number used
    if (run->p.ref_rechoose) first = std::max(first, rechoose_step(run));  // one reference throughout
    std::vector<double> S, E, Nr;
    for (const auto& h : run->hist)
        if (h.iter > first) { S.push_back(h.shift); E.push_back(h.enum_); Nr.push_back(h.nref); }
    out->first_step = first + 1;
    out->n_samples = (int64_t)S.size();
    if (S.size() < 16) return 0;
    double ms, es, me, mn, r, er, dummy;
    std::vector<double> ones(S.size(), 1.0);
    blocking(S, ones, ms, es, dummy, r, er);
    blocking(E, Nr, me, dummy, mn, r, er);
    out->shift = eref + ms;
    out->shift_err = es;
    out->e_proj = (eref + run->hproj) + r;
    out->e_proj_err = er;
    out->converged = std::fabs(out->shift - out->e_proj) < run->p.conv_tol && es < run->p.conv_tol &&
                     er < run->p.conv_tol;
    return 0;
}

int fciqmc_get_walkers(const fciqmc_run* run, uint64_t* dets, double* vals, int64_t cap, int64_t* n) {
    if (!run || !run->eng || !n) return fail(FCIQMC_EINVAL, "null argument");
    std::vector<uint64_t> ab;
    std::vector<double> v;
    CHECK(run->eng->get_walkers(ab, v));
    *n = (int64_t)v.size();
    if (*n > cap) return fail(FCIQMC_EOVERFLOW, "need room for %lld determinants", (long long)*n);
    if (*n > 0) {
        if (!dets || !vals) return fail(FCIQMC_EINVAL, "null output array");
        std::memcpy(dets, ab.data(), sizeof(uint64_t) * ab.size());
        std::memcpy(vals, v.data(), sizeof(double) * v.size());
    }
    return 0;
}

int fciqmc_set_walkers(fciqmc_run* run, const uint64_t* dets, const double* vals, int64_t n) {
    if (!run || !run->eng) return fail(FCIQMC_ESTATE, "run not initialised");
    if (n < 0 || (n > 0 && (!dets || !vals))) return fail(FCIQMC_EINVAL, "bad walker arrays");
    std::vector<std::pair<uint64_t, uint64_t>> keys((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        if (!valid_det(run->sys, dets[2 * i], dets[2 * i + 1]))
            return fail(FCIQMC_EINVAL, "entry %lld is not a valid determinant", (long long)i);
        const double v = vals[i];
        if (!(v != 0.0) || !std::isfinite(v)) return fail(FCIQMC_EINVAL, "entry %lld has a zero or non-finite value", (long long)i);
        if (run->p.mode == FCIQMC_MODE_INTEGER && (v != std::floor(v) || std::fabs(v) > 2e9))
            return fail(FCIQMC_EINVAL, "integer mode needs integral values (entry %lld)", (long long)i);
        keys[(size_t)i] = {dets[2 * i], dets[2 * i + 1]};
    }
    std::sort(keys.begin(), keys.end());
    if (std::adjacent_find(keys.begin(), keys.end()) != keys.end()) return fail(FCIQMC_EINVAL, "duplicate determinants");
    CHECK(run->eng->set_walkers(dets, vals, n));
    const int64_t A = run->p.shift_interval;
    run->t_set = run->t;
    run->nw_ring[(size_t)(run->t % (A + 1))] = run->eng->last_nw();
    return 0;
}

int fciqmc_set_core(fciqmc_run* run, int64_t n_core, int64_t* n_out) {
    if (!run || !run->eng) return fail(FCIQMC_ESTATE, "run not initialised");
    if (run->batch) return fail(FCIQMC_ESTATE, "the run belongs to a batch");
    if (run->p.mode != FCIQMC_MODE_REAL)
        return fail(FCIQMC_EINVAL, "the semi-stochastic projection needs real coefficients");
    if (run->p.adaptive_shift)
        return fail(FCIQMC_EINVAL, "the adaptive shift and a deterministic space are not combined");
    if (n_core < 0 || n_core > kMaxCore)
        return fail(FCIQMC_EINVAL, "n_core must be in [0, %lld]", (long long)kMaxCore);
    CHECK(run->eng->set_core(n_core));
    if (n_out) *n_out = run->eng->core_size();
    return 0;
}

int fciqmc_get_core(const fciqmc_run* run, uint64_t* dets, int64_t capacity, int64_t* n_out, int64_t* nnz_out) {
    if (!run || !run->eng) return fail(FCIQMC_ESTATE, "run not initialised");
    const int64_t n = run->eng->core_size();
    if (n_out) *n_out = n;
    if (nnz_out) *nnz_out = run->eng->core_nnz();
    if (dets && capacity > 0) {
        const auto& c = run->eng->core_dets();
        const int64_t m = std::min(n, capacity);
        std::copy(c.begin(), c.begin() + 2 * m, dets);
    }
    return 0;
}

int fciqmc_get_core_row(const fciqmc_run* run, int64_t k, int32_t* cols, double* vals, int64_t cap, int64_t* n_out) {
    if (!run || !run->eng) return fail(FCIQMC_ESTATE, "run not initialised");
    CHECK(run->eng->core_row(k, cols, vals, cap, n_out));
    return 0;
}

int fciqmc_get_reference(const fciqmc_run* run, uint64_t* alpha, uint64_t* beta, double* e_ref) {
    if (!run) return fail(FCIQMC_EINVAL, "null argument");
    if (alpha) *alpha = run->proj_a;
    if (beta) *beta = run->proj_b;
    if (e_ref) *e_ref = (run->h00 + run->sys->e_core) + run->hproj;
    return 0;
}

int fciqmc_get_checkpoint(const fciqmc_run* run, fciqmc_checkpoint* out) {
    if (!run || !out) return fail(FCIQMC_EINVAL, "null argument");
    out->iter = run->t;
    out->shift = run->S;
    out->vary_shift = run->vary;
    out->last_update_iter = run->t_last;
    out->last_update_nw = run->nw_last;
    return 0;
}

int fciqmc_set_checkpoint(fciqmc_run* run, const fciqmc_checkpoint* in) {
    if (!run || !in) return fail(FCIQMC_EINVAL, "null argument");
    if (in->iter < 0) return fail(FCIQMC_EINVAL, "negative iteration");
    const int64_t A = run->p.shift_interval;
    const double nw0 = run->nw_ring[(size_t)(run->t % (A + 1))];
    run->t = in->iter;
    run->t_set = in->iter;
    run->nw_ring[(size_t)(run->t % (A + 1))] = nw0;
    run->S = in->shift;
    run->vary = in->vary_shift ? 1 : 0;
    run->t_last = in->last_update_iter;
    run->nw_last = in->last_update_nw;
    run->t_vary = run->vary ? in->last_update_iter : -1;
    run->hist.clear();
    return 0;
}

int fciqmc_matrix_elements(const fciqmc_system* sys, const uint64_t* di, const uint64_t* dj, int64_t n,
                           double* out) {
    if (!sys || (n > 0 && (!di || !dj || !out))) return fail(FCIQMC_EINVAL, "null argument");
    if (n == 0) return 0;
    for (int64_t i = 0; i < n; ++i)
        if (!valid_det(sys, di[2 * i], di[2 * i + 1]) || !valid_det(sys, dj[2 * i], dj[2 * i + 1]))
            return fail(FCIQMC_EINVAL, "pair %lld holds an invalid determinant", (long long)i);
    Arena tmp;
    uint64_t *a = nullptr, *b = nullptr;
    double* o = nullptr;
    CHECK(dalloc(tmp, &a, (size_t)n * 2));
    CHECK(dalloc(tmp, &b, (size_t)n * 2));
    CHECK(dalloc(tmp, &o, (size_t)n));
    HIP_OK(hipMemcpy(a, di, sizeof(uint64_t) * 2 * n, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(b, dj, sizeof(uint64_t) * 2 * n, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_hij, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, 0,
                       sys->view(), a, b, (long long)n, o);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpy(out, o, sizeof(double) * n, hipMemcpyDeviceToHost));
    tmp.clear();
    return 0;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Matrix elements without allocation: the staging of the pairs and of the
// results lives in one statically sized device array instead of buffers
// allocated per call.  Each device holds its own copy of the array (for the
// life of the process); host code must use the address hipGetSymbolAddress
// returns for it on that device, never the array's name, which on the host
// is only a stand-in.  Layout: kNoAllocPairs determinant pairs of
// (alpha, beta) words for D_i, the same for D_j, then kNoAllocPairs results.
// ---------------------------------------------------------------------------
namespace {
constexpr int64_t kNoAllocPairs = 1 << 16;
constexpr size_t kNoAllocBytes = (size_t)kNoAllocPairs * (4 * sizeof(uint64_t) + sizeof(double));
constexpr int kMaxDevices = 64;
std::mutex g_scratch_lock;               // one call at a time uses a device's array
char* g_scratch_ptr[kMaxDevices] = {};   // its device address, per device
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
// Device address of `scratch` on device dev (which must be current), looked
// up once per device.  Called with g_scratch_lock held.
int scratch_on(int dev, char** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(FCIQMC_EDEVICE, "device %d out of range", dev);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(FCIQMC_EDEVICE, "no device address for the scratch array");
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[dev];
    return 0;
}
// Restores the caller's current device when it goes out of scope.
struct DeviceGuard {
    int prev = -1;
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};
}  // namespace

extern "C" int fciqmc_pchb_row(const fciqmc_system* csys, int opp, int64_t row, double* prob, int32_t* alias,
                               double* weight, double* sum) {
    if (!csys || !prob || !alias || !weight || !sum) return fail(FCIQMC_EINVAL, "null argument");
    fciqmc_system* sys = const_cast<fciqmc_system*>(csys);
    const int64_t N = sys->N;
    const int64_t K = opp ? N * N : N * (N - 1) / 2;
    if (row < 0 || row >= K) return fail(FCIQMC_EINVAL, "row %lld out of range [0, %lld)", (long long)row, (long long)K);
    CHECK(build_pchb(sys, nullptr));
    std::vector<uint64_t> h((size_t)K);
    const size_t at = (size_t)row * (size_t)K;
    HIP_OK(hipMemcpy(h.data(), (opp ? sys->hb_opp : sys->hb_same) + at, sizeof(uint64_t) * K, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(prob, (opp ? sys->hbp_opp : sys->hbp_same) + at, sizeof(double) * K, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(sum, (opp ? sys->hb_sum_opp : sys->hb_sum_same) + row, sizeof(double), hipMemcpyDeviceToHost));
    // the weights from the integrals, as the construction forms them: row
    // (I alpha, J beta) or I < J; column (A, B) ordered, or A < B in
    // lexicographic order
    auto eri = [&](int64_t p, int64_t q, int64_t r, int64_t t) {
        auto tri = [](int64_t x, int64_t y) { return x >= y ? x * (x + 1) / 2 + y : y * (y + 1) / 2 + x; };
        const int64_t X = tri(p, q), Y = tri(r, t);
        return sys->eri_host[(size_t)tri(X, Y)];
    };
    auto pair = [N](int64_t k, int64_t& x, int64_t& y) {
        for (x = 0; k >= N - 1 - x; ++x) k -= N - 1 - x;
        y = x + 1 + k;
    };
    int64_t I, J;
    if (opp) { I = row / N; J = row % N; } else pair(row, I, J);
    for (int64_t c = 0; c < K; ++c) {
        alias[c] = (int32_t)(h[(size_t)c] & ((1u << kHbAliasBits) - 1u));
        int64_t A, B;
        if (opp) { A = c / N; B = c % N; } else pair(c, A, B);
        double v;
        if (opp) v = (A == I || B == J) ? 0.0 : eri(A, I, B, J);
        else v = (A == I || A == J || B == I || B == J) ? 0.0 : eri(A, I, B, J) - eri(A, J, B, I);
        weight[c] = std::fabs(v);
    }
    return 0;
}

extern "C" int fciqmc_matrix_elements_noalloc(const fciqmc_system* sys, const uint64_t* di, const uint64_t* dj,
                                              int64_t n, double* out) {
    if (!sys || (n > 0 && (!di || !dj || !out))) return fail(FCIQMC_EINVAL, "null argument");
    if (n < 0) return fail(FCIQMC_EINVAL, "n must be >= 0");
    if (n > kNoAllocPairs)
        return fail(FCIQMC_EINVAL, "n = %lld exceeds the %lld pairs the allocation-free call stages",
                    (long long)n, (long long)kNoAllocPairs);
    if (n == 0) return 0;
    for (int64_t i = 0; i < n; ++i)
        if (!valid_det(sys, di[2 * i], di[2 * i + 1]) || !valid_det(sys, dj[2 * i], dj[2 * i + 1]))
            return fail(FCIQMC_EINVAL, "pair %lld holds an invalid determinant", (long long)i);
    std::lock_guard<std::mutex> lock(g_scratch_lock);
    DeviceGuard guard;
    HIP_OK(hipGetDevice(&guard.prev));
    HIP_OK(hipSetDevice(sys->device));
    char* base = nullptr;
    CHECK(scratch_on(sys->device, &base));
    uint64_t* a = reinterpret_cast<uint64_t*>(base);
    uint64_t* b = a + 2 * kNoAllocPairs;
    double* o = reinterpret_cast<double*>(b + 2 * kNoAllocPairs);
    HIP_OK(hipMemcpy(a, di, sizeof(uint64_t) * 2 * n, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(b, dj, sizeof(uint64_t) * 2 * n, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_hij, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, 0,
                       sys->view(), a, b, (long long)n, o);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpy(out, o, sizeof(double) * n, hipMemcpyDeviceToHost));
    return 0;
}

// ---------------------------------------------------------------------------
// Replica pairs and the second-order correction from discarded spawns
// (Sec. "Perturbative correction", Eq. (pt2_correction)).
// ---------------------------------------------------------------------------
struct fciqmc_pair {
    fciqmc_run* r[2] = {nullptr, nullptr};
    bool fixed[2] = {false, false};  // the runs' own bucket-growth setting, restored on free
    Arena arena;
    double* part = nullptr;  // per-bucket partial sums
    int64_t part_n = 0;
    double* res = nullptr;   // per paired step of a call: PT2 sum, overlap
    int64_t res_n = 0;
    unsigned* err = nullptr;
    hipEvent_t ev = nullptr;  // the pair kernels queued so far on the first replica's stream are done
    std::vector<double> num;  // per paired step: 1/dtau^2 sum S^1 S^2 / (E_0 - H_jj) (NaN: not evaluated)
    std::vector<double> ovl;  // and the replica overlap of the populations it began from
    // replica 2-RDM: the accumulated matrix (M x M over spin-orbital pairs)
    // and each replica's population table of the step being sampled
    bool rdm = false;
    double* G = nullptr;
    int64_t M = 0;
    int64_t rdm_steps = 0;
    uint64_t* tkeys[2] = {nullptr, nullptr};
    double* tvals[2] = {nullptr, nullptr};
    int32_t* tused[2] = {nullptr, nullptr};
    int64_t tslots[2] = {0, 0};
    ~fciqmc_pair() {
        if (ev) (void)hipEventDestroy(ev);
        arena.clear();
    }
};

void pair_detach(fciqmc_run* run) {
    fciqmc_pair* p = run->pair;
    for (auto& x : p->r)
        if (x == run) x = nullptr;
    run->pair = nullptr;
}

namespace {
int log2_of(int64_t x) {
    int k = 0;
    while ((int64_t)1 << (k + 1) <= x) ++k;
    return k;
}
// Queue both sums of a paired step over the two replicas on the first
// replica's stream, after both have stepped: the overlap of the
// populations the step started from and the discarded-spawn sum; their
// values land in out[1] and out[0] (device memory).  The replicas may hold
// different bucket counts (a store that grew during the step); the launch
// covers the larger count.  No host wait here: the kernel reads the second
// replica's records and previous store, which its next merge overwrites,
// and that merge comes only after the host has waited for the first
// replica's next step, queued behind this kernel on the same stream.
template <int W, class V> void launch_pair_sums(fciqmc_pair* p, int64_t B1, int64_t B2, double e0, double* out,
                                                hipStream_t s) {
    const EngineBase* a = p->r[0]->eng.get();
    const EngineBase* b = p->r[1]->eng.get();
    const Store<V> s1 = *static_cast<const Store<V>*>(a->previous_store());
    const Store<V> s2 = *static_cast<const Store<V>*>(b->previous_store());
    const int64_t Bm = std::max(B1, B2);
    const int sh1 = log2_of(Bm) - log2_of(B1), sh2 = log2_of(Bm) - log2_of(B2);
    hipLaunchKernelGGL((k_pair_sums<W, V>), dim3((unsigned)std::min<int64_t>(Bm, 4096)), dim3(kThreads), 0, s,
                       p->r[0]->sys->view(), s1, sh1, s2, sh2, a->bucket_entries(),
                       (const Rec<W, V>*)a->rej_records(), a->rej_offsets(), a->rej_counts(),
                       (const Rec<W, V>*)b->rej_records(), b->rej_offsets(), b->rej_counts(), (int)Bm, e0,
                       p->r[0]->h00, p->part, p->part + Bm, p->err);
    hipLaunchKernelGGL(k_sum2, dim3(1), dim3(kThreads), 0, s, p->part, p->part + Bm, (int)Bm, out);
}
int pair_sums(fciqmc_pair* p, double e0, double* out) {
    fciqmc_run* a = p->r[0];
    const int64_t B1 = a->eng->buckets(), B2 = p->r[1]->eng->buckets();
    const int64_t Bm = std::max(B1, B2);
    if (p->part_n < 2 * Bm) {
        HIP_OK(hipStreamSynchronize(a->stream));  // queued pair kernels still use the old buffer
        p->arena.release(p->part);
        p->part = nullptr;
        CHECK(dalloc(p->arena, &p->part, (size_t)(2 * Bm)));
        p->part_n = 2 * Bm;
    }
    const int k = a->eng->kind();
    if (k == 0) launch_pair_sums<1, int32_t>(p, B1, B2, e0, out, a->stream);
    else if (k == 1) launch_pair_sums<1, double>(p, B1, B2, e0, out, a->stream);
    else if (k == 2) launch_pair_sums<2, int32_t>(p, B1, B2, e0, out, a->stream);
    else launch_pair_sums<2, double>(p, B1, B2, e0, out, a->stream);
    HIP_OK(hipGetLastError());
    return 0;
}
// One paired step's sample of the replica 2-RDM, queued on the first
// replica's stream after both have stepped (and before either steps
// again): tables of both populations the step started from, the exact
// diagonal terms, and each replica's generated excitations against the
// other's table.  n_tau: each population's size at tau.
template <int W, class V> int launch_pair_rdm(fciqmc_pair* p, const int64_t n_tau[2], hipStream_t s) {
    const EngineBase* e[2] = {p->r[0]->eng.get(), p->r[1]->eng.get()};
    for (int i = 0; i < 2; ++i) {
        const int64_t want = (int64_t)next_pow2((uint64_t)std::max<int64_t>(256, 2 * n_tau[i]));
        if (want > p->tslots[i]) {
            HIP_OK(hipStreamSynchronize(s));  // queued samples still read the old tables
            p->arena.release(p->tkeys[i]);
            p->arena.release(p->tvals[i]);
            p->arena.release(p->tused[i]);
            p->tkeys[i] = nullptr;
            p->tvals[i] = nullptr;
            p->tused[i] = nullptr;
            p->tslots[i] = 0;
            CHECK(dalloc(p->arena, &p->tkeys[i], (size_t)want * W));
            CHECK(dalloc(p->arena, &p->tvals[i], (size_t)want));
            CHECK(dalloc(p->arena, &p->tused[i], (size_t)want));
            p->tslots[i] = want;
        }
    }
    PopTable<W> T[2];
    for (int i = 0; i < 2; ++i) {
        T[i].keys = p->tkeys[i];
        T[i].vals = p->tvals[i];
        T[i].used = p->tused[i];
        T[i].mask = (uint64_t)p->tslots[i] - 1;
        HIP_OK(hipMemsetAsync(p->tused[i], 0, sizeof(int32_t) * p->tslots[i], s));
        const Store<V> st = *static_cast<const Store<V>*>(e[i]->previous_store());
        const int B = (int)e[i]->buckets();
        hipLaunchKernelGGL((k_pop_table<W, V>), dim3((unsigned)std::min(B, 4096)), dim3(kThreads), 0, s, st,
                           e[i]->bucket_entries(), B, T[i]);
    }
    const int N = p->r[0]->sys->N;
    {
        const Store<V> s1 = *static_cast<const Store<V>*>(e[0]->previous_store());
        const int B = (int)e[0]->buckets();
        hipLaunchKernelGGL((k_rdm_diag<W, V>), dim3((unsigned)std::min(B, 1024)), dim3(kThreads),
                           sizeof(double) * (size_t)p->M, s, s1, e[0]->bucket_entries(), B, T[1], N, p->G);
    }
    for (int i = 0; i < 2; ++i) {
        const int64_t n = e[i]->rdm_count();
        if (n == 0) continue;
        hipLaunchKernelGGL((k_rdm_off<W>), dim3((unsigned)std::min<int64_t>((n + kThreads - 1) / kThreads, 8192)),
                           dim3(kThreads), 0, s, static_cast<const RdmRec<W>*>(e[i]->rdm_records()), n, T[1 - i], N,
                           p->G);
    }
    HIP_OK(hipGetLastError());
    p->rdm_steps += 1;
    return 0;
}
int pair_rdm(fciqmc_pair* p, const int64_t n_tau[2]) {
    const int k = p->r[0]->eng->kind();
    hipStream_t s = p->r[0]->stream;
    if (k == 0) return launch_pair_rdm<1, int32_t>(p, n_tau, s);
    if (k == 1) return launch_pair_rdm<1, double>(p, n_tau, s);
    if (k == 2) return launch_pair_rdm<2, int32_t>(p, n_tau, s);
    return launch_pair_rdm<2, double>(p, n_tau, s);
}
// Energy of a 2-RDM over spin-orbital pairs (the matrix made hermitian):
// sum_pq h_pq gamma_pq + sum_{k<l,m<n} Gamma_{kl,mn} <kl||mn>, divided by
// the norm trace / (n(n-1)/2), plus E_core; gamma_pq = sum_r Gamma_{pr,qr}/(n-1).
double rdm_energy(const fciqmc_system* sys, const std::vector<double>& G, double& norm) {
    const int N = sys->N, K = 2 * N, ne = sys->na + sys->nb;
    const int64_t M = (int64_t)K * (K - 1) / 2;
    auto P = [K](int k, int l) { return (int64_t)k * (2 * K - k - 1) / 2 + (l - k - 1); };
    auto eri = [&](int a, int b, int c, int d) {
        auto tri = [](int x, int y) { return x >= y ? x * (x + 1) / 2 + y : y * (y + 1) / 2 + x; };
        const int64_t X = tri(a, b), Y = tri(c, d);
        return sys->eri_host[(size_t)(X >= Y ? X * (X + 1) / 2 + Y : Y * (Y + 1) / 2 + X)];
    };
    double tr = 0.0;
    for (int64_t i = 0; i < M; ++i) tr = tr + G[(size_t)(i * M + i)];
    const double npair = (double)ne * (double)(ne - 1) / 2.0;
    norm = tr / npair;
    double e1 = 0.0;
    for (int p = 0; p < K; ++p)
        for (int q = 0; q < K; ++q) {
            if (p / N != q / N) continue;
            double g = 0.0;
            for (int r = 0; r < K; ++r) {
                if (r == p || r == q) continue;
                int a = p, b = r, c = q, d = r, sg = 1;
                if (a > b) { std::swap(a, b); sg = -sg; }
                if (c > d) { std::swap(c, d); sg = -sg; }
                const double v = G[(size_t)(P(a, b) * M + P(c, d))];
                g = g + (sg > 0 ? v : -v);
            }
            const double gam = g / (double)(ne - 1);
            const double x = sys->h1_host[(size_t)((p % N) * N + (q % N))] * gam;
            e1 = e1 + x;
        }
    double e2 = 0.0;
    for (int k = 0; k < K; ++k)
        for (int l = k + 1; l < K; ++l)
            for (int m = 0; m < K; ++m)
                for (int n = m + 1; n < K; ++n) {
                    const double v = G[(size_t)(P(k, l) * M + P(m, n))];
                    if (v == 0.0) continue;
                    const double d = (k / N == m / N && l / N == n / N) ? eri(k % N, m % N, l % N, n % N) : 0.0;
                    const double x = (k / N == n / N && l / N == m / N) ? eri(k % N, n % N, l % N, m % N) : 0.0;
                    const double a = d - x;
                    const double c = v * a;
                    e2 = e2 + c;
                }
    const double e = e1 + e2;
    return e / norm + sys->e_core;
}
// Waits for a stream when it goes out of scope (also on an error return), so
// that no queued pair kernel outlives the call that queued it.
struct StreamWait {
    hipStream_t s;
    ~StreamWait() { (void)hipStreamSynchronize(s); }
};
}  // namespace

extern "C" {

int fciqmc_pair_create(fciqmc_run* r1, fciqmc_run* r2, fciqmc_pair** out) {
    if (!r1 || !r2 || !out || !r1->eng || !r2->eng) return fail(FCIQMC_EINVAL, "null argument");
    *out = nullptr;
    if (r1 == r2) return fail(FCIQMC_EINVAL, "a pair needs two runs");
    for (fciqmc_run* r : {r1, r2}) {
        if (r->batch) return fail(FCIQMC_ESTATE, "a run in a batch cannot join a pair");
        if (r->pair) return fail(FCIQMC_ESTATE, "the run already belongs to a pair");
    }
    if (r1->sys != r2->sys || r1->eng->kind() != r2->eng->kind() || r1->p.tau != r2->p.tau ||
        r1->ref_a != r2->ref_a || r1->ref_b != r2->ref_b)
        return fail(FCIQMC_EINVAL, "replicas need the same system, layout, time step and reference");
    if (r1->p.ref_rechoose || r2->p.ref_rechoose)
        return fail(FCIQMC_EINVAL, "replicas keep one reference: no re-choice (ref_rechoose)");
    if (r1->p.seed == r2->p.seed && r1->p.replica_id == r2->p.replica_id)
        return fail(FCIQMC_EINVAL, "replicas need different random streams (replica_id or seed)");
    std::unique_ptr<fciqmc_pair> p(new fciqmc_pair());
    CHECK(dalloc(p->arena, &p->err, 1));
    HIP_OK(hipEventCreateWithFlags(&p->ev, hipEventDisableTiming));
    const int64_t B = std::max(r1->eng->buckets(), r2->eng->buckets());
    fciqmc_run* rr[2] = {r1, r2};
    for (int i = 0; i < 2; ++i) {
        p->fixed[i] = rr[i]->eng->fixed_b;
        CHECK(rr[i]->eng->rebucket((int)B));
        rr[i]->eng->fixed_b = true;
        CHECK(rr[i]->eng->set_collect(true));
        p->r[i] = rr[i];
        rr[i]->pair = p.get();
    }
    *out = p.release();
    return 0;
}

int fciqmc_pair_step(fciqmc_pair* p, int n_steps, fciqmc_step_stats* stats1, fciqmc_step_stats* stats2,
                     double* de2) {
    if (!p) return fail(FCIQMC_EINVAL, "null argument");
    if (!p->r[0] || !p->r[1]) return fail(FCIQMC_ESTATE, "a replica of the pair was freed");
    if (n_steps < 0) return fail(FCIQMC_EINVAL, "n_steps must be >= 0");
    fciqmc_run* a = p->r[0];
    fciqmc_run* b = p->r[1];
    if (n_steps == 0) return 0;
    if (p->res_n < 2 * (int64_t)n_steps) {
        HIP_OK(hipStreamSynchronize(a->stream));
        p->arena.release(p->res);
        p->res = nullptr;
        CHECK(dalloc(p->arena, &p->res, (size_t)2 * n_steps));
        p->res_n = 2 * (int64_t)n_steps;
    }
    std::vector<char> has_ovl((size_t)n_steps, 0), has_num((size_t)n_steps, 0);
    int done = 0;  // steps whose values are queued (or skipped)
    auto steps = [&]() -> int {
        StreamWait wait{a->stream};
        HIP_OK(hipMemsetAsync(p->err, 0, sizeof(unsigned), a->stream));
        for (int i = 0; i < n_steps; ++i) {
            const double e0 = (a->S + b->S) / 2.0;  // the shifts this step uses
            const int64_t n_tau[2] = {a->eng->ndets(), b->eng->ndets()};
            HIP_OK(hipEventRecord(p->ev, a->stream));
            CHECK(fciqmc_step(a, 1, stats1 ? stats1 + i : nullptr));
            // the pair kernels of the last step read the second replica's
            // records and previous store: done before it steps (normally
            // already, since the host waited for the first replica's step
            // behind them)
            HIP_OK(hipEventSynchronize(p->ev));
            CHECK(fciqmc_step(b, 1, stats2 ? stats2 + i : nullptr));
            // every step is evaluated, also one in which a store outgrew its
            // buckets (the sums read each replica in its own layout)
            CHECK(pair_sums(p, e0, p->res + 2 * i));
            has_ovl[i] = 1;
            has_num[i] = 1;
            if (p->rdm) CHECK(pair_rdm(p, n_tau));
            done = i + 1;
            const int64_t Ba = a->eng->buckets(), Bb = b->eng->buckets();
            if (Ba != Bb) {
                // both use the larger count from the next step on; the sums
                // just queued read the records and stores that re-bucketing
                // replaces, so they finish first
                HIP_OK(hipStreamSynchronize(a->stream));
                const int64_t B = std::max(Ba, Bb);
                CHECK(a->eng->rebucket((int)B));
                CHECK(b->eng->rebucket((int)B));
            }
        }
        return 0;
    };
    const int rc = steps();  // the queued pair kernels have finished when it returns
    // the values of the steps done (all of them, or those before an error)
    std::vector<double> h((size_t)2 * n_steps, NAN);
    unsigned e = 0;
    if (done > 0) {
        HIP_OK(hipMemcpy(h.data(), p->res, sizeof(double) * 2 * done, hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(&e, p->err, sizeof(unsigned), hipMemcpyDeviceToHost));
    }
    for (int i = 0; i < n_steps; ++i) {
        double num = NAN, ovl = NAN;
        if (i < done) {
            num = has_num[i] ? h[2 * i] / (a->p.tau * a->p.tau) : NAN;
            ovl = has_ovl[i] ? h[2 * i + 1] : NAN;
            if (!e) {
                p->num.push_back(num);
                p->ovl.push_back(ovl);
            }
        }
        if (de2) de2[i] = num / ovl;
    }
    if (rc) return rc;
    if (e) return fail(FCIQMC_EDEVICE, "pair sums: an LDS hash claim did not complete");
    return 0;
}

int fciqmc_pair_rdm_enable(fciqmc_pair* p, int on) {
    if (!p) return fail(FCIQMC_EINVAL, "null argument");
    if (!p->r[0] || !p->r[1]) return fail(FCIQMC_ESTATE, "a replica of the pair was freed");
    if (!on) {
        p->rdm = false;
        CHECK(p->r[0]->eng->set_rdm(false));
        CHECK(p->r[1]->eng->set_rdm(false));
        return 0;
    }
    const int64_t K = 2 * (int64_t)p->r[0]->sys->N;
    const int64_t M = K * (K - 1) / 2;
    hipStream_t s = p->r[0]->stream;
    HIP_OK(hipStreamSynchronize(s));
    if (!p->G || p->M != M) {
        p->arena.release(p->G);
        p->G = nullptr;
        CHECK(dalloc(p->arena, &p->G, (size_t)(M * M)));
        p->M = M;
    }
    HIP_OK(hipMemsetAsync(p->G, 0, sizeof(double) * M * M, s));
    HIP_OK(hipStreamSynchronize(s));
    p->rdm_steps = 0;
    CHECK(p->r[0]->eng->set_rdm(true));
    CHECK(p->r[1]->eng->set_rdm(true));
    p->rdm = true;
    return 0;
}

int fciqmc_pair_rdm(const fciqmc_pair* cp, double* gamma, int64_t capacity, int64_t* dim, double* e_var,
                    double* norm, int64_t* steps) {
    if (!cp) return fail(FCIQMC_EINVAL, "null argument");
    fciqmc_pair* p = const_cast<fciqmc_pair*>(cp);
    if (!p->r[0]) return fail(FCIQMC_ESTATE, "a replica of the pair was freed");
    if (!p->G) return fail(FCIQMC_ESTATE, "the pair has not sampled a 2-RDM (fciqmc_pair_rdm_enable)");
    const int64_t M = p->M;
    if (dim) *dim = M;
    if (steps) *steps = p->rdm_steps;
    HIP_OK(hipStreamSynchronize(p->r[0]->stream));
    std::vector<double> G((size_t)(M * M));
    HIP_OK(hipMemcpy(G.data(), p->G, sizeof(double) * M * M, hipMemcpyDeviceToHost));
    // hermitian part: the two orderings of a sampled pair carry independent noise
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = i + 1; j < M; ++j) {
            const double x = G[(size_t)(i * M + j)] + G[(size_t)(j * M + i)];
            const double h = x * 0.5;
            G[(size_t)(i * M + j)] = h;
            G[(size_t)(j * M + i)] = h;
        }
    double nm = 0.0;
    const double e = p->rdm_steps > 0 ? rdm_energy(p->r[0]->sys, G, nm) : NAN;
    if (e_var) *e_var = e;
    if (norm) *norm = nm;
    if (gamma) {
        if (capacity < M * M) return fail(FCIQMC_EOVERFLOW, "gamma needs %lld entries", (long long)(M * M));
        std::memcpy(gamma, G.data(), sizeof(double) * M * M);
    }
    return 0;
}

int fciqmc_pair_pt2(const fciqmc_pair* p, int64_t skip, double* mean, double* err, int64_t* n) {
    if (!p || !mean || !err || !n) return fail(FCIQMC_EINVAL, "null argument");
    std::vector<double> x, y;
    for (size_t i = (size_t)std::max<int64_t>(skip, 0); i < p->num.size(); ++i)
        if (!std::isnan(p->num[i]) && !std::isnan(p->ovl[i])) { x.push_back(p->num[i]); y.push_back(p->ovl[i]); }
    *n = (int64_t)x.size();
    *mean = NAN;
    *err = NAN;
    if (x.empty()) return 0;
    double mx, ex, my, r, er;
    if (x.size() < 16) {
        mx = 0.0; my = 0.0;
        for (size_t i = 0; i < x.size(); ++i) { mx += x[i]; my += y[i]; }
        *mean = my != 0.0 ? mx / my : NAN;
        return 0;
    }
    blocking(x, y, mx, ex, my, r, er);
    *mean = r;
    *err = er;
    return 0;
}

void fciqmc_pair_free(fciqmc_pair* p) {
    if (!p) return;
    for (int i = 0; i < 2; ++i) {
        fciqmc_run* r = p->r[i];
        if (!r) continue;
        (void)r->eng->set_collect(false);
        r->eng->fixed_b = p->fixed[i];
        r->pair = nullptr;
    }
    delete p;
}

}  // extern "C"
