// capi.cpp -- the extern "C" boundary: argument checks, error codes, the
// per-thread error message, and hipGraph recording of comparison calls.

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <sstream>

#include "ops.h"
#include "bluestein.h"
#include "persist.h"

namespace bc {
GraphCache::~GraphCache() {
    for (auto &kv : entries) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
        for (void *p : kv.second.blocks) (void)hipFree(p);
    }
}
}  // namespace bc

using namespace bc;

namespace {

thread_local std::string tl_err;

struct StreamScope {
    hipStream_t prev;
    explicit StreamScope(void *s) : prev(tl_stream) { tl_stream = (hipStream_t)s; }
    ~StreamScope() { tl_stream = prev; }
};

template <class F>
int guard(F &&f) {
    try {
        f();
        return BC_OK;
    } catch (const Error &e) {
        tl_err = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        tl_err = "host allocation failed";
        return BC_ERR_OOM;
    } catch (const std::exception &e) {
        tl_err = e.what();
        return BC_ERR_ARG;
    }
}

void check_ctx(const bc_ctx *c) { BC_REQUIRE(c, BC_ERR_ARG, "null context"); }

// Drops one owner of the context; the last one waits for the device and
// deletes it.
void ctx_release(bc_ctx *c) {
    if (!c || c->refs.fetch_sub(1) != 1) return;
    (void)hipDeviceSynchronize();
    delete c;
}
void check_keys(const bc_ctx *c, const bc_keys *k) {
    BC_REQUIRE(k, BC_ERR_ARG, "null keys");
    BC_REQUIRE(k->ctx == c, BC_ERR_PARAM, "keys belong to another context");
}

// Every stage kind of the persistent executor exists for this context: fp64
// arithmetic, single-pass transforms and 2^13-word transform blocks.
bool persist_supported(const bc_ctx *c) {
    return use_fp64(c) && c->ntt_single_pass && c->logN - ntt_parts_log(c) == 13 && c->ntt_chunk_bytes == 0;
}

// Installs a recorder on the calling thread for one scope.
struct RecordScope {
    Recorder *prev;
    explicit RecordScope(Recorder *r) : prev(tl_rec) { tl_rec = r; }
    ~RecordScope() { tl_rec = prev; }
};

// Runs the comparison and copies results into the caller's buffers.
void run_compare(bc_ctx *c, const bc_keys *k, int ndig, const CtB *A, const CtB *B, const bc_ctb *lt_out,
                 const bc_ctb *max_out, const bc_ctb *min_out, hipStream_t st, int circuit = BC_CIRCUIT_UNIVARIATE) {
    bool mm = max_out || min_out;
    CompareResult r = compare(c, k, ndig, A, B, mm, st, circuit);
    const int G = A[0].count;
    if (lt_out) copy_ct(c, r.lt, from_abi(c, lt_out), st);
    for (int d = 0; d < ndig; d++) {
        if (max_out) copy_ct(c, r.mx.slice(d * G, G, c->N), from_abi(c, &max_out[d]), st);
        if (min_out) copy_ct(c, r.mn.slice(d * G, G, c->N), from_abi(c, &min_out[d]), st);
    }
}

// At least n library streams on context c (workspace tags of its slices),
// and their events; the caller holds c->split_mu.
void ensure_split_streams(bc_ctx *c, int n) {
    while ((int)c->split_streams.size() < n) {
        hipStream_t s;
        hipEvent_t e;
        BC_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        c->split_streams.push_back(s);
        BC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        c->split_done.push_back(e);
    }
    if (!c->split_fork) BC_HIP(hipEventCreateWithFlags(&c->split_fork, hipEventDisableTiming));
}

// Slices of one comparison for the persistent executor: the groups split
// into S slices (S = the device's XCDs, at most the group count); slice s
// is lane lane0 + s of `rec`, pinned to XCD s, its workspace tagged with c's
// library stream s.  Before the launch `origin` must wait for those streams'
// earlier work (join_before), after it they wait for the launch
// (join_after).  The caller holds c->split_mu and has run ensure_split_streams.
int record_slices(bc_ctx *c, const bc_keys *k, int ndig, const CtB *A, const CtB *B, const bc_ctb *lt_out,
                  const bc_ctb *max_out, const bc_ctb *min_out, Recorder &rec, int lane0) {
    const int G = A[0].count, S = std::min(rec.nq, G);
    auto cut = [&](const bc_ctb *x, int lo, int cnt) {
        bc_ctb sl = *x;
        sl.data = x->data + (size_t)lo * bc_ct_words(c, x->level, x->ncomp);
        sl.count = cnt;
        return sl;
    };
    RecordScope rs(&rec);
    for (int i = 0; i < S; i++) {
        const int lo = (int)((int64_t)G * i / S), hi = (int)((int64_t)G * (i + 1) / S);
        std::vector<CtB> a(ndig), b(ndig);
        std::vector<bc_ctb> mx, mn;
        for (int d = 0; d < ndig; d++) {
            a[d] = A[d].slice(lo, hi - lo, c->N);
            b[d] = B[d].slice(lo, hi - lo, c->N);
            if (max_out) mx.push_back(cut(&max_out[d], lo, hi - lo));
            if (min_out) mn.push_back(cut(&min_out[d], lo, hi - lo));
        }
        bc_ctb lt;
        if (lt_out) lt = cut(lt_out, lo, hi - lo);
        rec.lane = lane0 + i;
        if ((int)rec.lane_xcd.size() <= rec.lane) rec.lane_xcd.resize(rec.lane + 1, 0);
        rec.lane_xcd[rec.lane] = i;
        StreamScope sc(c->split_streams[i]);
        run_compare(c, k, ndig, a.data(), b.data(), lt_out ? &lt : nullptr, max_out ? mx.data() : nullptr,
                    min_out ? mn.data() : nullptr, c->split_streams[i]);
    }
    return S;
}
void join_before(bc_ctx *c, int S, hipStream_t origin) {
    for (int i = 0; i < S; i++) {
        BC_HIP(hipEventRecord(c->split_done[i], c->split_streams[i]));
        BC_HIP(hipStreamWaitEvent(origin, c->split_done[i], 0));
    }
}
void join_after(bc_ctx *c, int S, hipStream_t origin) {
    BC_HIP(hipEventRecord(c->split_fork, origin));
    for (int i = 0; i < S; i++) BC_HIP(hipStreamWaitEvent(c->split_streams[i], c->split_fork, 0));
}

// The comparison as one persistent launch on `origin`, one lane per XCD.
void run_compare_persistent(bc_ctx *c, const bc_keys *k, int ndig, const CtB *A, const CtB *B, const bc_ctb *lt_out,
                            const bc_ctb *max_out, const bc_ctb *min_out, hipStream_t origin) {
    BC_REQUIRE(persist_supported(c), BC_ERR_ARG, "persistent mode: unsupported context");
    std::lock_guard<std::mutex> lk(c->split_mu);
    if (!c->runner) c->runner.reset(new PersistRunner());
    c->runner->check_stall();
    Recorder rec;
    rec.nq = persist_xcds();
    ensure_split_streams(c, rec.nq);
    const int S = std::min(rec.nq, A[0].count);
    join_before(c, S, origin);
    record_slices(c, k, ndig, A, B, lt_out, max_out, min_out, rec, 0);
    c->runner->run(c, rec, origin);
    join_after(c, S, origin);
}

// run_compare with the groups split over ctx->split library streams (when
// the batch has that many groups): forked from `origin` by an event, each
// branch compares its slice of every plane into its slice of every output,
// and `origin` waits for every branch.  Independent branches let one slice's
// compute-bound kernels overlap another's memory-bound ones.
void run_compare_split(bc_ctx *c, const bc_keys *k, int ndig, const CtB *A, const CtB *B, const bc_ctb *lt_out,
                       const bc_ctb *max_out, const bc_ctb *min_out, hipStream_t origin) {
    const int G = A[0].count, n = std::min(c->split, G);
    if (c->persistent && c->exec_mode != BC_EXEC_PER_OP) {
        run_compare_persistent(c, k, ndig, A, B, lt_out, max_out, min_out, origin);
        return;
    }
    if (n <= 1) {
        run_compare(c, k, ndig, A, B, lt_out, max_out, min_out, origin);
        return;
    }
    std::lock_guard<std::mutex> lk(c->split_mu);
    while ((int)c->split_streams.size() < n) {
        hipStream_t s;
        hipEvent_t e;
        BC_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        c->split_streams.push_back(s);
        BC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        c->split_done.push_back(e);
    }
    if (!c->split_fork) BC_HIP(hipEventCreateWithFlags(&c->split_fork, hipEventDisableTiming));
    BC_HIP(hipEventRecord(c->split_fork, origin));
    auto cut = [&](const bc_ctb *x, int lo, int cnt) {
        bc_ctb s = *x;
        s.data = x->data + (size_t)lo * bc_ct_words(c, x->level, x->ncomp);
        s.count = cnt;
        return s;
    };
    for (int i = 0; i < n; i++) {
        const int lo = (int)((int64_t)G * i / n), hi = (int)((int64_t)G * (i + 1) / n);
        std::vector<CtB> a(ndig), b(ndig);
        std::vector<bc_ctb> mx, mn;
        for (int d = 0; d < ndig; d++) {
            a[d] = A[d].slice(lo, hi - lo, c->N);
            b[d] = B[d].slice(lo, hi - lo, c->N);
            if (max_out) mx.push_back(cut(&max_out[d], lo, hi - lo));
            if (min_out) mn.push_back(cut(&min_out[d], lo, hi - lo));
        }
        bc_ctb lt;
        if (lt_out) lt = cut(lt_out, lo, hi - lo);
        hipStream_t s = c->split_streams[i];
        BC_HIP(hipStreamWaitEvent(s, c->split_fork, 0));
        {
            StreamScope sc(s);
            run_compare(c, k, ndig, a.data(), b.data(), lt_out ? &lt : nullptr, max_out ? mx.data() : nullptr,
                        min_out ? mn.data() : nullptr, s);
        }
        BC_HIP(hipEventRecord(c->split_done[i], s));
        BC_HIP(hipStreamWaitEvent(origin, c->split_done[i], 0));
    }
}

// Token of a key set inside a graph key (keys are identified by their unique
// id, never by address).
std::string keys_token(const bc_keys *k) { return "|K" + std::to_string(k->uid) + "|"; }

std::string graph_key(int ndig, const bc_ctb *a, const bc_ctb *b, const bc_ctb *lt, const bc_ctb *mx,
                      const bc_ctb *mn, void *st, const bc_keys *k) {
    std::ostringstream os;
    os << ndig << '|' << st << keys_token(k);
    auto put = [&](const bc_ctb *x) { os << '|' << (x ? (void *)x->data : nullptr) << ',' << (x ? x->count : 0) << ','
                                        << (x ? x->level : 0); };
    for (int d = 0; d < ndig; d++) {
        put(&a[d]);
        put(&b[d]);
        put(mx ? &mx[d] : nullptr);
        put(mn ? &mn[d] : nullptr);
    }
    put(lt);
    return os.str();
}

// Checks one comparison request and returns its planes and the levels and
// noise estimates of its outputs (BC_ERR_LEVEL, before anything is launched,
// when the circuit does not fit the chain).
CircuitNoise check_compare(bc_ctx *ctx, const bc_keys *keys, int ndigits, const bc_ctb *a_digits,
                           const bc_ctb *b_digits, const bc_ctb *lt_out, const bc_ctb *max_out,
                           const bc_ctb *min_out, std::vector<CtB> &A, std::vector<CtB> &B,
                           int circuit = BC_CIRCUIT_UNIVARIATE) {
    check_ctx(ctx);
    check_keys(ctx, keys);
    BC_REQUIRE(a_digits && b_digits && ndigits >= 1 && ndigits <= 16, BC_ERR_ARG, "bad digit planes");
    BC_REQUIRE(lt_out || max_out || min_out, BC_ERR_ARG, "no output requested");
    A.clear();
    B.clear();
    double in_noise = 0;
    for (int d = 0; d < ndigits; d++) {
        A.push_back(from_abi(ctx, &a_digits[d]));
        B.push_back(from_abi(ctx, &b_digits[d]));
        in_noise = std::max(in_noise, std::max(A.back().noise, B.back().noise));
    }
    for (int d = 0; d < ndigits; d++) {
        BC_REQUIRE(A[d].count == A[0].count && B[d].count == A[0].count, BC_ERR_ARG,
                   "every plane needs the same count");
        BC_REQUIRE(A[d].level == A[0].level && B[d].level == A[0].level, BC_ERR_ARG,
                   "every plane needs the same level");
        BC_REQUIRE(A[d].ncomp == 2 && B[d].ncomp == 2, BC_ERR_ARG, "planes must have 2 components");
    }
    CircuitNoise cn{};
    compare_levels(ctx->noise, A[0].level, in_noise, ndigits, max_out || min_out, &cn, circuit);
    auto want = [&](const bc_ctb *x, int lv) {
        CtB o = from_abi(ctx, x);
        BC_REQUIRE(o.count == A[0].count && o.level == lv && o.ncomp == 2, BC_ERR_ARG,
                   "output batch: wrong count, level or components");
    };
    if (lt_out) want(lt_out, cn.lt_level);
    for (int d = 0; d < ndigits; d++) {
        if (max_out) want(&max_out[d], cn.mm_level);
        if (min_out) want(&min_out[d], cn.mm_level);
    }
    return cn;
}

// Records the output estimates in the caller's batch descriptors.
void set_compare_noise(const CircuitNoise &cn, int ndigits, bc_ctb *lt_out, bc_ctb *max_out, bc_ctb *min_out) {
    if (lt_out) lt_out->noise_bits = (float)cn.lt_noise;
    for (int d = 0; d < ndigits; d++) {
        if (max_out) max_out[d].noise_bits = (float)cn.mm_noise;
        if (min_out) min_out[d].noise_bits = (float)cn.mm_noise;
    }
}

}  // namespace

struct bc_group {
    std::vector<bc_ctx *> ctxs;
    std::vector<hipStream_t> streams;  // one per member (default priority)
    std::vector<hipEvent_t> done;      // one per member
    hipEvent_t fork = nullptr;
    hipStream_t cap = nullptr;          // recording stream
    bc::GraphCache graphs;
    std::mutex mu;
    int mode = BC_GROUP_FORK_JOIN;
    std::unique_ptr<bc::PersistRunner> runner;  // persistent mode's upload and launch state
    hipEvent_t joined = nullptr;
    ~bc_group() {
        if (joined) (void)hipEventDestroy(joined);
        for (auto s : streams) (void)hipStreamDestroy(s);
        for (auto e : done) (void)hipEventDestroy(e);
        if (fork) (void)hipEventDestroy(fork);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

extern "C" {

int bc_group_create(int32_t n, bc_ctx *const *ctxs, bc_group **out) {
    return guard([&] {
        BC_REQUIRE(n >= 1 && n <= 16 && ctxs && out, BC_ERR_ARG, "bad group");
        std::unique_ptr<bc_group> g(new bc_group());
        for (int i = 0; i < n; i++) {
            check_ctx(ctxs[i]);
            for (int j = 0; j < i; j++) BC_REQUIRE(ctxs[j] != ctxs[i], BC_ERR_ARG, "a context appears twice");
            g->ctxs.push_back(ctxs[i]);
            hipStream_t s;
            BC_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
            g->streams.push_back(s);
            hipEvent_t e;
            BC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            g->done.push_back(e);
        }
        BC_HIP(hipEventCreateWithFlags(&g->fork, hipEventDisableTiming));
        BC_HIP(hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking));
        BC_HIP(hipEventCreateWithFlags(&g->joined, hipEventDisableTiming));
        g->runner.reset(new PersistRunner());
        g->mode = BC_GROUP_FORK_JOIN;
        for (bc_ctx *c : g->ctxs) c->refs.fetch_add(1);  // released by bc_group_destroy
        *out = g.release();
    });
}

int bc_group_destroy(bc_group *g) {
    return guard([&] {
        if (!g) return;
        (void)hipDeviceSynchronize();
        const std::vector<bc_ctx *> members = g->ctxs;
        delete g;
        for (bc_ctx *c : members) ctx_release(c);
    });
}

int bc_group_set_mode(bc_group *g, int32_t mode) {
    return guard([&] {
        BC_REQUIRE(g, BC_ERR_ARG, "null group");
        BC_REQUIRE(mode == BC_GROUP_FORK_JOIN || mode == BC_GROUP_PERSISTENT, BC_ERR_ARG, "unknown group mode");
        if (mode == BC_GROUP_PERSISTENT)
            for (bc_ctx *c : g->ctxs)
                BC_REQUIRE(persist_supported(c), BC_ERR_ARG,
                           "persistent mode needs N = 2^13..2^15, primes below 2^50 and the default transform schedule");
        std::lock_guard<std::mutex> lk(g->mu);
        g->mode = mode;
    });
}

int bc_group_get_mode(const bc_group *g, int32_t *mode, int32_t *stages, int32_t *tickets, int32_t *workgroups) {
    return guard([&] {
        BC_REQUIRE(g, BC_ERR_ARG, "null group");
        if (mode) *mode = g->mode;
        if (stages) *stages = g->runner->last.stages;
        if (tickets) *tickets = g->runner->last.tickets;
        if (workgroups) *workgroups = g->runner->last.grid;
    });
}

int bc_group_compare(bc_group *g, const bc_keys *const *keys, const int32_t *ndigits, const bc_ctb *const *a_digits,
                     const bc_ctb *const *b_digits, bc_ctb *const *lt_out, bc_ctb *const *max_out,
                     bc_ctb *const *min_out, void *stream) {
    return guard([&] {
        BC_REQUIRE(g && keys && ndigits && a_digits && b_digits, BC_ERR_ARG, "null argument");
        const int n = (int)g->ctxs.size();
        std::vector<std::vector<CtB>> A(n), B(n);
        std::vector<CircuitNoise> cns;
        std::ostringstream key;
        for (int i = 0; i < n; i++) {
            const bc_ctb *lt = lt_out ? lt_out[i] : nullptr, *mx = max_out ? max_out[i] : nullptr,
                         *mn = min_out ? min_out[i] : nullptr;
            cns.push_back(check_compare(g->ctxs[i], keys[i], ndigits[i], a_digits[i], b_digits[i], lt, mx, mn, A[i],
                                        B[i]));
            key << graph_key(ndigits[i], a_digits[i], b_digits[i], lt, mx, mn, stream, keys[i]) << '#';
        }
        for (int i = 0; i < n; i++)
            set_compare_noise(cns[i], ndigits[i], lt_out ? lt_out[i] : nullptr, max_out ? max_out[i] : nullptr,
                              min_out ? min_out[i] : nullptr);
        hipStream_t st = (hipStream_t)stream;
        std::lock_guard<std::mutex> lk(g->mu);
        g->runner->check_stall();
        const bool persist = g->mode == BC_GROUP_PERSISTENT;
        if (persist) key << "persistent";
        auto it = g->graphs.entries.find(key.str());
        if (it != g->graphs.entries.end()) {
            BC_HIP(hipGraphLaunch(it->second.exec, st));
            return;
        }
        // persistent mode: every member's launches recorded as one lane each
        // persistent mode: every member's groups split into one slice per
        // XCD, each slice a lane pinned to its XCD (lane i * kMaxXcd + s)
        const int nq = persist ? persist_xcds() : 1;
        std::vector<std::unique_lock<std::mutex>> member_locks;
        if (persist)
            for (bc_ctx *c : g->ctxs) {
                member_locks.emplace_back(c->split_mu);
                ensure_split_streams(c, nq);
            }
        auto record_all = [&](Recorder &rec) {
            rec.nq = nq;
            for (int i = 0; i < n; i++)
                record_slices(g->ctxs[i], keys[i], ndigits[i], A[i].data(), B[i].data(), lt_out ? lt_out[i] : nullptr,
                              max_out ? max_out[i] : nullptr, min_out ? min_out[i] : nullptr, rec, i * kMaxXcd);
        };
        if (persist) {
            // eager: the launch on `st` after the slices' earlier work; their
            // streams wait for it (their workspace blocks were used)
            for (int i = 0; i < n; i++) join_before(g->ctxs[i], std::min(nq, A[i][0].count), st);
            Recorder rec;
            record_all(rec);
            g->runner->run(g->ctxs[0], rec, st);
            for (int i = 0; i < n; i++) join_after(g->ctxs[i], std::min(nq, A[i][0].count), st);
            BC_HIP(hipStreamSynchronize(st));
            // recorded: the blocks the graph keeps, the table uploaded before
            // capture, the reset and the persistent launch captured
            for (auto *c : g->ctxs) {
                std::lock_guard<std::mutex> pg(c->pool.mu);
                c->pool.recording = true;
                c->pool.recorded.clear();
            }
            GraphEntry e;
            try {
                Recorder rec2;
                record_all(rec2);
                const PersistPlan plan2 = persist_plan(rec2);
                void *tab = nullptr;
                BC_HIP(hipMalloc(&tab, plan2.image.size()));
                e.blocks.push_back(tab);
                BC_HIP(hipMemcpy(tab, plan2.image.data(), plan2.image.size(), hipMemcpyHostToDevice));
                BC_HIP(hipStreamBeginCapture(g->cap, hipStreamCaptureModeRelaxed));
                try {
                    persist_run(plan2, tab, g->runner->stall, g->cap);
                } catch (...) {
                    hipGraph_t dead = nullptr;
                    (void)hipStreamEndCapture(g->cap, &dead);
                    if (dead) (void)hipGraphDestroy(dead);
                    throw;
                }
                BC_HIP(hipStreamEndCapture(g->cap, &e.graph));
                BC_HIP(hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0));
            } catch (...) {
                for (auto *c : g->ctxs) {
                    auto b = c->pool.detach_recorded();
                    e.blocks.insert(e.blocks.end(), b.begin(), b.end());
                }
                for (void *p : e.blocks) (void)hipFree(p);
                if (e.exec) (void)hipGraphExecDestroy(e.exec);
                if (e.graph) (void)hipGraphDestroy(e.graph);
                throw;
            }
            for (auto *c : g->ctxs) {
                auto b = c->pool.detach_recorded();
                e.blocks.insert(e.blocks.end(), b.begin(), b.end());
            }
            g->graphs.entries.emplace(key.str(), std::move(e));
            return;
        }
        // fork/join over the member streams; `origin` is the stream the
        // branches fork from and join back into
        auto run_all = [&](hipStream_t origin) {
            BC_HIP(hipEventRecord(g->fork, origin));
            for (int i = 0; i < n; i++) {
                BC_HIP(hipStreamWaitEvent(g->streams[i], g->fork, 0));
                StreamScope sc(g->streams[i]);
                run_compare(g->ctxs[i], keys[i], ndigits[i], A[i].data(), B[i].data(), lt_out ? lt_out[i] : nullptr,
                            max_out ? max_out[i] : nullptr, min_out ? min_out[i] : nullptr, g->streams[i]);
                BC_HIP(hipEventRecord(g->done[i], g->streams[i]));
                BC_HIP(hipStreamWaitEvent(origin, g->done[i], 0));
            }
        };
        run_all(st);  // eager: results of this call; warms every pool
        BC_HIP(hipStreamSynchronize(st));
        for (auto *c : g->ctxs) {
            std::lock_guard<std::mutex> pg(c->pool.mu);
            c->pool.recording = true;
            c->pool.recorded.clear();
        }
        GraphEntry e;
        BC_HIP(hipStreamBeginCapture(g->cap, hipStreamCaptureModeRelaxed));
        try {
            run_all(g->cap);
        } catch (...) {
            hipGraph_t dead = nullptr;
            (void)hipStreamEndCapture(g->cap, &dead);
            if (dead) (void)hipGraphDestroy(dead);
            for (auto *c : g->ctxs) {
                std::lock_guard<std::mutex> pg(c->pool.mu);
                c->pool.recording = false;
                c->pool.recorded.clear();
            }
            throw;
        }
        BC_HIP(hipStreamEndCapture(g->cap, &e.graph));
        BC_HIP(hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0));
        for (auto *c : g->ctxs) {
            auto b = c->pool.detach_recorded();
            e.blocks.insert(e.blocks.end(), b.begin(), b.end());
        }
        g->graphs.entries.emplace(key.str(), std::move(e));
    });
}

const char *bc_strerror(int code) {
    switch (code) {
        case BC_OK: return "ok";
        case BC_ERR_ARG: return "invalid argument";
        case BC_ERR_PARAM: return "invalid or mismatched parameters";
        case BC_ERR_LEVEL: return "out of levels or noise budget";
        case BC_ERR_OOM: return "out of memory";
        case BC_ERR_HIP: return "HIP runtime error";
        case BC_ERR_KEY: return "missing switching key";
        default: return "unknown error";
    }
}

const char *bc_last_error(void) { return tl_err.c_str(); }

int bc_noise_estimate(const bc_params *prm, int32_t op, int32_t level, double a_bits, double b_bits,
                      double *out_bits) {
    return guard([&] {
        BC_REQUIRE(prm && out_bits, BC_ERR_ARG, "null argument");
        const NoiseModel m(*prm, param_moduli(*prm));
        BC_REQUIRE(level >= 0 && level < prm->nQ, BC_ERR_ARG, "level out of range");
        const double a = m.input((float)a_bits), b = m.input((float)b_bits);
        double r = 0;
        switch (op) {
            case BC_NOISE_FRESH: r = m.fresh(); break;
            case BC_NOISE_BUDGET: r = m.budget(level); break;
            case BC_NOISE_ADD: r = m.add(a, b); break;
            case BC_NOISE_TENSOR: r = m.tensor(a, b); break;
            case BC_NOISE_MUL:
                r = m.product(level, a, b, -INFINITY);
                m.require(level, r, "multiplication");
                if (level > 0) r = m.mod_switch(level, r);
                break;
            case BC_NOISE_MOD_SWITCH:
                BC_REQUIRE(level >= 1, BC_ERR_LEVEL, "modulus switch: no prime left to drop at level 0");
                r = m.mod_switch(level, a);
                break;
            case BC_NOISE_ROTATE: r = m.rotate(level, a); break;
            default: throw Error(BC_ERR_ARG, "unknown noise operation");
        }
        *out_bits = r;
    });
}

int bc_noise_compare_circuit(const bc_params *prm, int32_t circuit, int32_t in_level, double in_bits,
                             int32_t ndigits, double *lt_bits, double *maxmin_bits, int32_t *lt_level,
                             int32_t *maxmin_level) {
    return guard([&] {
        BC_REQUIRE(prm, BC_ERR_ARG, "null argument");
        BC_REQUIRE(in_level >= 0 && in_level < prm->nQ && ndigits >= 1 && ndigits <= 16, BC_ERR_ARG,
                   "bad level or digit count");
        const NoiseModel m(*prm, param_moduli(*prm));
        CircuitNoise cn{};
        compare_levels(m, in_level, m.input((float)in_bits), ndigits, maxmin_bits != nullptr, &cn, circuit);
        if (lt_bits) *lt_bits = cn.lt_noise;
        if (maxmin_bits) *maxmin_bits = cn.mm_noise;
        if (lt_level) *lt_level = cn.lt_level;
        if (maxmin_level) *maxmin_level = cn.mm_level;
    });
}

int bc_noise_compare(const bc_params *prm, int32_t in_level, double in_bits, int32_t ndigits, double *lt_bits,
                     double *maxmin_bits) {
    return bc_noise_compare_circuit(prm, BC_CIRCUIT_UNIVARIATE, in_level, in_bits, ndigits, lt_bits, maxmin_bits,
                                    nullptr, nullptr);
}

int bc_ctx_create(const bc_params *prm, bc_ctx **out) {
    return guard([&] {
        BC_REQUIRE(prm && out, BC_ERR_ARG, "null argument");
        std::unique_ptr<bc_ctx> c(new bc_ctx());
        build_context(c.get(), *prm);
        c->graphs.reset(new GraphCache());
        // set-up of the allocation-free entry point on this device (a failed
        // lookup only disables that entry point)
        BC_HIP(hipGetDevice(&c->device));
        try {
            c->scratch = scratch_lookup(c->device);
        } catch (const Error &e) {
            c->scratch_err = e.what();
        }
        *out = c.release();
    });
}

int bc_ctx_destroy(bc_ctx *ctx) {
    return guard([&] { ctx_release(ctx); });
}

int bc_ctx_moduli(const bc_ctx *ctx, uint64_t *moduli, int32_t cap) {
    return guard([&] {
        check_ctx(ctx);
        BC_REQUIRE(moduli && cap >= ctx->nmod, BC_ERR_ARG, "moduli buffer too small");
        std::memcpy(moduli, ctx->mod.data(), sizeof(uint64_t) * ctx->nmod);
    });
}

int bc_ctx_slots(const bc_ctx *ctx) { return ctx ? ctx->M : BC_ERR_ARG; }

size_t bc_ct_words(const bc_ctx *ctx, int32_t level, int32_t ncomp) {
    if (!ctx || level < 0 || level >= ctx->nQ || ncomp < 1 || ncomp > 3) return 0;
    return (size_t)ncomp * (level + 1) * ctx->N;
}

size_t bc_ctx_pool_bytes(const bc_ctx *ctx) { return ctx ? ctx->pool.held : 0; }

int bc_ctx_trim(bc_ctx *ctx) {
    return guard([&] {
        check_ctx(ctx);
        ctx->pool.trim();
    });
}

int bc_keygen_rand_sizes(const bc_ctx *ctx, int32_t nrot, size_t *n_words, size_t *n_errors) {
    return guard([&] {
        check_ctx(ctx);
        BC_REQUIRE(nrot >= 0 && n_words && n_errors, BC_ERR_ARG, "bad arguments");
        *n_words = (size_t)ctx->nQ * ctx->N + (size_t)(1 + nrot) * ctx->dnum * ctx->nmod * ctx->N;
        *n_errors = (size_t)ctx->N + (size_t)(1 + nrot) * ctx->dnum * ctx->N;
    });
}

int bc_keygen(bc_ctx *ctx, const int8_t *s, const uint64_t *a_words, const int32_t *errors, const int32_t *rot_steps,
              int32_t nrot, bc_keys **out) {
    return guard([&] {
        check_ctx(ctx);
        BC_REQUIRE(out, BC_ERR_ARG, "null output");
        StreamScope sc(nullptr);
        *out = keygen(ctx, s, a_words, errors, rot_steps, nrot);
        ctx->refs.fetch_add(1);
    });
}

int bc_keys_destroy(bc_keys *keys) {
    return guard([&] {
        if (!keys) return;
        (void)hipDeviceSynchronize();
        // graphs recorded with these keys hold their device pointers: drop
        // them (group graphs are keyed by the same unique id and never match
        // a later key set)
        bc_ctx *c = keys->ctx;
        const std::string tok = keys_token(keys);
        {
            std::lock_guard<std::mutex> g(c->graph_mu);
            auto &ents = c->graphs->entries;
            for (auto it = ents.begin(); it != ents.end();) {
                if (it->first.find(tok) != std::string::npos) {
                    if (it->second.exec) (void)hipGraphExecDestroy(it->second.exec);
                    if (it->second.graph) (void)hipGraphDestroy(it->second.graph);
                    for (void *p : it->second.blocks) (void)hipFree(p);
                    it = ents.erase(it);
                } else {
                    ++it;
                }
            }
        }
        delete keys;
        ctx_release(c);
    });
}

int bc_keys_export(bc_ctx *ctx, const bc_keys *keys, void *buf, size_t cap, size_t *size) {
    return guard([&] {
        check_ctx(ctx);
        check_keys(ctx, keys);
        BC_REQUIRE(size, BC_ERR_ARG, "null size");
        StreamScope sc(nullptr);
        *size = keys_export(ctx, keys, buf, cap);
    });
}

int bc_keys_import(bc_ctx *ctx, const void *buf, size_t size, bc_keys **out) {
    return guard([&] {
        check_ctx(ctx);
        BC_REQUIRE(out, BC_ERR_ARG, "null output");
        StreamScope sc(nullptr);
        *out = keys_import(ctx, buf, size);
        ctx->refs.fetch_add(1);
    });
}

int bc_encrypt(bc_ctx *ctx, const bc_keys *keys, const uint32_t *slots, const int8_t *u, const int32_t *errors,
               bc_ctb *out, void *stream) {
    return guard([&] {
        check_ctx(ctx);
        check_keys(ctx, keys);
        BC_REQUIRE(out && out->data && out->count >= 1, BC_ERR_ARG, "bad output batch");
        out->level = ctx->nQ - 1;
        out->ncomp = 2;
        StreamScope sc(stream);
        encrypt(ctx, keys, slots, u, errors, from_abi(ctx, out), (hipStream_t)stream);
        out->noise_bits = (float)ctx->noise.fresh();
    });
}

namespace {
// After a synchronising read-back: a persistent launch of this context that
// stalled (its results invalid) is reported here as well as by the next launch.
void report_stall(bc_ctx *c) {
    std::lock_guard<std::mutex> lk(c->split_mu);
    if (c->runner) c->runner->check_stall();
}
}  // namespace

int bc_decrypt_poly(bc_ctx *ctx, const bc_keys *keys, const bc_ctb *in, uint32_t *coeffs, void *stream) {
    return guard([&] {
        check_ctx(ctx);
        check_keys(ctx, keys);
        BC_REQUIRE(coeffs, BC_ERR_ARG, "null output");
        StreamScope sc(stream);
        decrypt_poly(ctx, keys, from_abi(ctx, in), coeffs, (hipStream_t)stream);
        report_stall(ctx);
    });
}

int bc_decrypt(bc_ctx *ctx, const bc_keys *keys, const bc_ctb *in, uint32_t *slots, void *stream) {
    return guard([&] {
        check_ctx(ctx);
        check_keys(ctx, keys);
        BC_REQUIRE(slots, BC_ERR_ARG, "null output");
        StreamScope sc(stream);
        CtB x = from_abi(ctx, in);
        std::vector<uint32_t> coeffs((size_t)x.count * ctx->N);
        decrypt_poly(ctx, keys, x, coeffs.data(), (hipStream_t)stream);
        report_stall(ctx);
        decode_slots(ctx, coeffs.data(), slots, x.count);
    });
}

int bc_export(bc_ctx *ctx, const bc_ctb *in, uint64_t *host, void *stream) {
    return guard([&] {
        check_ctx(ctx);
        StreamScope sc(stream);
        export_ct(ctx, from_abi(ctx, in), host, (hipStream_t)stream);
        report_stall(ctx);
    });
}

int bc_import(bc_ctx *ctx, const uint64_t *host, bc_ctb *out, void *stream) {
    return guard([&] {
        check_ctx(ctx);
        StreamScope sc(stream);
        import_ct(ctx, host, from_abi(ctx, out), (hipStream_t)stream);
    });
}

int bc_tensor(bc_ctx *ctx, const bc_ctb *a, const bc_ctb *b, bc_ctb *out, void *stream) {
    return guard([&] {
        check_ctx(ctx);
        StreamScope sc(stream);
        const CtB x = from_abi(ctx, a), y = from_abi(ctx, b), o = from_abi(ctx, out);
        const double nb = ctx->noise.tensor(x.noise, y.noise);
        ctx->noise.require(o.level, nb, "tensor");
        tensor(ctx, x, y, o, (hipStream_t)stream);
        out->noise_bits = (float)nb;
    });
}

int bc_relin(bc_ctx *ctx, const bc_keys *keys, const bc_ctb *in, bc_ctb *out, void *stream) {
    return guard([&] {
        check_ctx(ctx);
        check_keys(ctx, keys);
        StreamScope sc(stream);
        const CtB x = from_abi(ctx, in), o = from_abi(ctx, out);
        const double nb = ctx->noise.key_switch(x.level, x.noise);
        ctx->noise.require(x.level, nb, "relinearisation");
        relin(ctx, keys, x, o, (hipStream_t)stream);
        out->noise_bits = (float)nb;
    });
}

int bc_mod_switch(bc_ctx *ctx, const bc_ctb *in, bc_ctb *out, void *stream) {
    return guard([&] {
        check_ctx(ctx);
        StreamScope sc(stream);
        const CtB x = from_abi(ctx, in);
        BC_REQUIRE(x.level >= 1, BC_ERR_LEVEL, "modulus switch: no prime left to drop at level 0");
        const CtB o = from_abi(ctx, out);
        const double nb = ctx->noise.mod_switch(x.level, x.noise);
        ctx->noise.require(x.level, x.noise, "modulus switch input");
        mod_switch(ctx, x, o, (hipStream_t)stream);
        out->noise_bits = (float)nb;
    });
}

int bc_mul_relin(bc_ctx *ctx, const bc_keys *keys, const bc_ctb *a, const bc_ctb *b, bc_ctb *out, void *stream) {
    return guard([&] {
        check_ctx(ctx);
        check_keys(ctx, keys);
        StreamScope sc(stream);
        const CtB x = from_abi(ctx, a), y = from_abi(ctx, b), o = from_abi(ctx, out);
        const int lv = std::min(x.level, y.level);
        double nb = ctx->noise.product(lv, x.noise, y.noise, -INFINITY);
        ctx->noise.require(lv, nb, "multiplication");
        if (lv > 0) nb = ctx->noise.mod_switch(lv, nb);
        mul_relin(ctx, keys, x, y, o, (hipStream_t)stream);
        out->noise_bits = (float)nb;
    });
}

int bc_mul_relin_noalloc(bc_ctx *ctx, const bc_keys *keys, const bc_ctb *a, const bc_ctb *b, bc_ctb *out,
                         void *stream) {
    return guard([&] {
        check_ctx(ctx);
        check_keys(ctx, keys);
        BC_REQUIRE(ctx->scratch, BC_ERR_HIP, "allocation-free workspace unavailable: " + ctx->scratch_err);
        int dev = -1;
        BC_HIP(hipGetDevice(&dev));
        BC_REQUIRE(dev == ctx->device, BC_ERR_ARG, "allocation-free call on another device than the context's");
        StreamScope sc(stream);
        const CtB x = from_abi(ctx, a), y = from_abi(ctx, b), o = from_abi(ctx, out);
        const int lv = std::min(x.level, y.level);
        const size_t need = mul_relin_workspace(ctx, x.count, lv);
        BC_REQUIRE(need <= kScratchBytes, BC_ERR_ARG,
                   "allocation-free multiplication needs " + std::to_string(need) + " bytes of workspace; the fixed " +
                       "scratch holds " + std::to_string(kScratchBytes) + " (use fewer ciphertexts per call)");
        double nb = ctx->noise.product(lv, x.noise, y.noise, -INFINITY);
        ctx->noise.require(lv, nb, "multiplication");
        if (lv > 0) nb = ctx->noise.mod_switch(lv, nb);
        ArenaScope ws(ctx->scratch, kScratchBytes);
        mul_relin(ctx, keys, x, y, o, (hipStream_t)stream);
        out->noise_bits = (float)nb;
    });
}

int bc_rotate(bc_ctx *ctx, const bc_keys *keys, const bc_ctb *in, int32_t steps, bc_ctb *out, void *stream) {
    return guard([&] {
        check_ctx(ctx);
        check_keys(ctx, keys);
        StreamScope sc(stream);
        const CtB x = from_abi(ctx, in), o = from_abi(ctx, out);
        const double nb = ctx->noise.rotate(x.level, x.noise);
        ctx->noise.require(x.level, nb, "rotation");
        rotate(ctx, keys, x, steps, o, (hipStream_t)stream);
        out->noise_bits = (float)nb;
    });
}

int bc_add(bc_ctx *ctx, const bc_ctb *a, const bc_ctb *b, bc_ctb *out, void *stream) {
    return guard([&] {
        check_ctx(ctx);
        StreamScope sc(stream);
        const CtB x = from_abi(ctx, a), y = from_abi(ctx, b), o = from_abi(ctx, out);
        const double nb = ctx->noise.add(x.noise, y.noise);
        ctx->noise.require(o.level, nb, "addition");
        add_sub(ctx, x, y, o, false, (hipStream_t)stream);
        out->noise_bits = (float)nb;
    });
}

int bc_sub(bc_ctx *ctx, const bc_ctb *a, const bc_ctb *b, bc_ctb *out, void *stream) {
    return guard([&] {
        check_ctx(ctx);
        StreamScope sc(stream);
        const CtB x = from_abi(ctx, a), y = from_abi(ctx, b), o = from_abi(ctx, out);
        const double nb = ctx->noise.add(x.noise, y.noise);
        ctx->noise.require(o.level, nb, "subtraction");
        add_sub(ctx, x, y, o, true, (hipStream_t)stream);
        out->noise_bits = (float)nb;
    });
}

int bc_mul_scalar(bc_ctx *ctx, const bc_ctb *a, int32_t c, bc_ctb *out, void *stream) {
    return guard([&] {
        check_ctx(ctx);
        StreamScope sc(stream);
        const CtB x = from_abi(ctx, a), o = from_abi(ctx, out);
        const double nb = ctx->noise.scalar(x.noise, (double)std::llabs(centred(ctx, c)));
        ctx->noise.require(o.level, nb, "scalar multiplication");
        mul_scalar(ctx, x, c, o, (hipStream_t)stream);
        out->noise_bits = (float)nb;
    });
}

int bc_add_const(bc_ctx *ctx, const bc_ctb *a, int32_t c, bc_ctb *out, void *stream) {
    return guard([&] {
        check_ctx(ctx);
        StreamScope sc(stream);
        const CtB x = from_abi(ctx, a), o = from_abi(ctx, out);
        const double nb = ctx->noise.add_const(x.noise);
        ctx->noise.require(o.level, nb, "constant addition");
        add_const(ctx, x, c, o, (hipStream_t)stream);
        out->noise_bits = (float)nb;
    });
}

int bc_compare_levels_circuit(const bc_ctx *ctx, int32_t circuit, int32_t in_level, int32_t ndigits,
                              int32_t *lt_level, int32_t *maxmin_level) {
    return guard([&] {
        check_ctx(ctx);
        BC_REQUIRE(in_level >= 0 && in_level < ctx->nQ && ndigits >= 1 && ndigits <= 16, BC_ERR_ARG,
                   "bad level or digit count");
        CircuitNoise cn{};
        compare_levels(ctx->noise, in_level, ctx->noise.fresh(), ndigits, false, &cn, circuit);
        if (lt_level) *lt_level = cn.lt_level;
        if (maxmin_level) *maxmin_level = cn.mm_level;
    });
}

int bc_compare_levels(const bc_ctx *ctx, int32_t in_level, int32_t ndigits, int32_t *lt_level, int32_t *maxmin_level) {
    return bc_compare_levels_circuit(ctx, BC_CIRCUIT_UNIVARIATE, in_level, ndigits, lt_level, maxmin_level);
}

int bc_packed_levels(const bc_ctx *ctx, int32_t circuit, int32_t in_level, int32_t digits_per_int, int32_t *lt_level) {
    return guard([&] {
        check_ctx(ctx);
        BC_REQUIRE(circuit == BC_CIRCUIT_UNIVARIATE || circuit == BC_CIRCUIT_BIVARIATE, BC_ERR_ARG, "unknown circuit");
        BC_REQUIRE(in_level >= 0 && in_level < ctx->nQ, BC_ERR_ARG, "bad level");
        BC_REQUIRE(digits_per_int >= 1 && (digits_per_int & (digits_per_int - 1)) == 0 &&
                       digits_per_int <= ctx->M / 2,
                   BC_ERR_ARG, "digits per integer must be a power of two up to half the slots");
        int lv = 0;
        double nb = 0;
        packed_levels(ctx->noise, in_level, ctx->noise.fresh(), digits_per_int, circuit, &lv, &nb);
        if (lt_level) *lt_level = lv;
    });
}

int bc_tournament_levels(const bc_ctx *ctx, int32_t circuit, int32_t in_level, int32_t window, int32_t *out_level) {
    return guard([&] {
        check_ctx(ctx);
        BC_REQUIRE(circuit == BC_CIRCUIT_UNIVARIATE || circuit == BC_CIRCUIT_BIVARIATE, BC_ERR_ARG, "unknown circuit");
        BC_REQUIRE(in_level >= 0 && in_level < ctx->nQ, BC_ERR_ARG, "bad level");
        BC_REQUIRE(window >= 1 && (window & (window - 1)) == 0 && window <= ctx->M / 2, BC_ERR_ARG,
                   "the window must be a power of two up to half the slots");
        int lv = 0;
        double nb = 0;
        tournament_levels(ctx->noise, in_level, ctx->noise.fresh(), window, circuit, &lv, &nb);
        if (out_level) *out_level = lv;
    });
}

namespace {
// BC_ERR_KEY unless `keys` hold rotation keys for steps 1, 2, 4, ... < len.
void require_shift_keys(const bc_keys *k, int len) {
    for (int s = 1; s < len; s *= 2) {
        bool have = false;
        for (int i = 0; i < k->ngal; i++) have = have || k->steps[i] == s;
        BC_REQUIRE(have, BC_ERR_KEY, "missing a rotation key for a shift of the packed schedule");
    }
}
}  // namespace

int bc_compare_packed(bc_ctx *ctx, const bc_keys *keys, int32_t circuit, int32_t digits_per_int, const bc_ctb *a,
                      const bc_ctb *b, bc_ctb *lt_out, void *stream) {
    return guard([&] {
        check_ctx(ctx);
        check_keys(ctx, keys);
        BC_REQUIRE(a && b && lt_out, BC_ERR_ARG, "null batch");
        const CtB x = from_abi(ctx, a), y = from_abi(ctx, b), o = from_abi(ctx, lt_out);
        BC_REQUIRE(x.count == y.count && x.level == y.level && x.ncomp == 2 && y.ncomp == 2, BC_ERR_ARG,
                   "packed operands: same count and level, 2 components");
        BC_REQUIRE(digits_per_int >= 1 && (digits_per_int & (digits_per_int - 1)) == 0 &&
                       digits_per_int <= ctx->M / 2,
                   BC_ERR_ARG, "digits per integer must be a power of two up to half the slots");
        int lv = 0;
        double nb = 0;
        packed_levels(ctx->noise, x.level, std::max(x.noise, y.noise), digits_per_int, circuit, &lv, &nb);
        BC_REQUIRE(o.count == x.count && o.level == lv && o.ncomp == 2, BC_ERR_ARG,
                   "output batch: wrong count, level or components");
        require_shift_keys(keys, digits_per_int);
        StreamScope sc(stream);
        const hipStream_t st = (hipStream_t)stream;
        const CtB r = compare_packed(ctx, keys, x, y, digits_per_int, circuit, st);
        copy_ct(ctx, r, o, st);
        lt_out->noise_bits = (float)nb;
    });
}

int bc_tournament(bc_ctx *ctx, const bc_keys *keys, int32_t circuit, int32_t window, int32_t want_max,
                  const bc_ctb *in, bc_ctb *out, void *stream) {
    return guard([&] {
        check_ctx(ctx);
        check_keys(ctx, keys);
        BC_REQUIRE(in && out, BC_ERR_ARG, "null batch");
        const CtB x = from_abi(ctx, in), o = from_abi(ctx, out);
        BC_REQUIRE(x.ncomp == 2, BC_ERR_ARG, "tournament input: 2 components");
        BC_REQUIRE(window >= 1 && (window & (window - 1)) == 0 && window <= ctx->M / 2, BC_ERR_ARG,
                   "the window must be a power of two up to half the slots");
        int lv = 0;
        double nb = 0;
        tournament_levels(ctx->noise, x.level, x.noise, window, circuit, &lv, &nb);
        BC_REQUIRE(o.count == x.count && o.level == lv && o.ncomp == 2, BC_ERR_ARG,
                   "output batch: wrong count, level or components");
        require_shift_keys(keys, window);
        StreamScope sc(stream);
        const hipStream_t st = (hipStream_t)stream;
        const CtB r = tournament(ctx, keys, x, window, want_max != 0, circuit, st);
        copy_ct(ctx, r, o, st);
        out->noise_bits = (float)nb;
    });
}

int bc_fpd_info(const bc_ctx *ctx, int32_t *degree, int32_t *nsteps, int32_t *steps, int32_t cap) {
    return guard([&] {
        check_ctx(ctx);
        const std::vector<int> st = frobenius_steps(ctx);
        if (degree) *degree = ctx->N / ctx->M;
        if (nsteps) *nsteps = (int32_t)st.size();
        if (steps) {
            BC_REQUIRE(cap >= (int32_t)st.size(), BC_ERR_ARG, "steps array too small");
            for (size_t i = 0; i < st.size(); i++) steps[i] = st[i];
        }
    });
}

int bc_encode_fpd(const bc_ctx *ctx, const uint32_t *elems, int32_t count, uint32_t *coeffs) {
    return guard([&] {
        check_ctx(ctx);
        BC_REQUIRE(elems && coeffs && count >= 1, BC_ERR_ARG, "encode: null buffer or empty batch");
        encode_fpd(ctx, elems, count, coeffs);
    });
}

int bc_decode_fpd(const bc_ctx *ctx, const uint32_t *coeffs, int32_t count, uint32_t *elems) {
    return guard([&] {
        check_ctx(ctx);
        BC_REQUIRE(elems && coeffs && count >= 1, BC_ERR_ARG, "decode: null buffer or empty batch");
        decode_fpd(ctx, coeffs, count, elems);
    });
}

int bc_encrypt_poly(bc_ctx *ctx, const bc_keys *keys, const uint32_t *coeffs, const int8_t *u, const int32_t *errors,
                    bc_ctb *out, void *stream) {
    return guard([&] {
        check_ctx(ctx);
        check_keys(ctx, keys);
        BC_REQUIRE(out && out->data && out->count >= 1, BC_ERR_ARG, "bad output batch");
        out->level = ctx->nQ - 1;
        out->ncomp = 2;
        StreamScope sc(stream);
        encrypt_poly(ctx, keys, coeffs, u, errors, from_abi(ctx, out), (hipStream_t)stream);
        out->noise_bits = (float)ctx->noise.fresh();
    });
}

int bc_extract_digits(bc_ctx *ctx, const bc_keys *keys, const bc_ctb *in, const int32_t *digits, int32_t ndigits,
                      bc_ctb *out, void *stream) {
    return guard([&] {
        check_ctx(ctx);
        check_keys(ctx, keys);
        BC_REQUIRE(in && out, BC_ERR_ARG, "null batch");
        const CtB x = from_abi(ctx, in), o = from_abi(ctx, out);
        // each doubling adds a rotated copy: the noise doubles and gains the key switch
        double nb = x.noise;
        for (size_t i = 0; i < frobenius_steps(ctx).size(); i++) nb = ctx->noise.add(nb, ctx->noise.rotate(x.level, nb));
        const int64_t dinv = centred(ctx, (int64_t)h_invmod((u64)((ctx->N / ctx->M) % ctx->p), (u64)ctx->p));
        nb = ctx->noise.scalar(nb, (double)std::llabs(dinv));
        ctx->noise.require(x.level, nb, "digit extraction");
        StreamScope sc(stream);
        std::vector<int> dg(digits ? digits : nullptr, digits ? digits + std::max(ndigits, 0) : nullptr);
        extract_digits(ctx, keys, x, dg.data(), (int)dg.size(), o, (hipStream_t)stream);
        out->noise_bits = (float)nb;
    });
}

int bc_bluestein_create(int32_t m, int32_t nprimes, int32_t bits, bc_bluestein **out) {
    return guard([&] {
        BC_REQUIRE(out, BC_ERR_ARG, "null output");
        *out = bluestein_create(m, nprimes, bits);
    });
}

int bc_bluestein_destroy(bc_bluestein *plan) {
    return guard([&] {
        if (plan) bluestein_destroy(plan);
    });
}

int bc_bluestein_info(const bc_bluestein *plan, int32_t *n, int32_t *conv_len, uint64_t *moduli) {
    return guard([&] {
        BC_REQUIRE(plan, BC_ERR_ARG, "null plan");
        int nn = 0, L = 0;
        bluestein_info(plan, &nn, &L, moduli);
        if (n) *n = nn;
        if (conv_len) *conv_len = L;
    });
}

int bc_bluestein_forward(bc_bluestein *plan, const uint64_t *in, uint64_t *out, int32_t count, void *stream) {
    return guard([&] {
        BC_REQUIRE(plan, BC_ERR_ARG, "null plan");
        BC_REQUIRE(in != out, BC_ERR_ARG, "the transform does not run in place");
        bluestein_forward(plan, in, out, count, (hipStream_t)stream);
    });
}

int bc_bluestein_inverse(bc_bluestein *plan, const uint64_t *in, uint64_t *out, int32_t count, void *stream) {
    return guard([&] {
        BC_REQUIRE(plan, BC_ERR_ARG, "null plan");
        BC_REQUIRE(in != out, BC_ERR_ARG, "the transform does not run in place");
        bluestein_inverse(plan, in, out, count, (hipStream_t)stream);
    });
}

int bc_compare_bivariate(bc_ctx *ctx, const bc_keys *keys, int32_t ndigits, const bc_ctb *a_digits,
                         const bc_ctb *b_digits, bc_ctb *lt_out, bc_ctb *max_out, bc_ctb *min_out, void *stream) {
    return guard([&] {
        std::vector<CtB> A, B;
        const CircuitNoise cn = check_compare(ctx, keys, ndigits, a_digits, b_digits, lt_out, max_out, min_out, A, B,
                                              BC_CIRCUIT_BIVARIATE);
        set_compare_noise(cn, ndigits, lt_out, max_out, min_out);
        StreamScope sc(stream);
        run_compare(ctx, keys, ndigits, A.data(), B.data(), lt_out, max_out, min_out, (hipStream_t)stream,
                    BC_CIRCUIT_BIVARIATE);
    });
}

int bc_set_exec_mode(bc_ctx *ctx, int32_t mode) {
    return guard([&] {
        check_ctx(ctx);
        BC_REQUIRE(mode == BC_EXEC_BATCHED || mode == BC_EXEC_GRAPH || mode == BC_EXEC_PER_OP, BC_ERR_ARG,
                   "unknown execution mode");
        ctx->exec_mode = mode;
    });
}

int bc_compare_max_min(bc_ctx *ctx, const bc_keys *keys, int32_t ndigits, const bc_ctb *a_digits,
                       const bc_ctb *b_digits, bc_ctb *lt_out, bc_ctb *max_out, bc_ctb *min_out, void *stream) {
    return guard([&] {
        std::vector<CtB> A, B;
        const CircuitNoise cn = check_compare(ctx, keys, ndigits, a_digits, b_digits, lt_out, max_out, min_out, A, B);
        set_compare_noise(cn, ndigits, lt_out, max_out, min_out);
        hipStream_t st = (hipStream_t)stream;
        StreamScope sc(stream);
        if (ctx->exec_mode != BC_EXEC_GRAPH || ctx->persistent) {  // a persistent call is one launch already
            run_compare_split(ctx, keys, ndigits, A.data(), B.data(), lt_out, max_out, min_out, st);
            return;
        }
        std::string key = graph_key(ndigits, a_digits, b_digits, lt_out, max_out, min_out, stream, keys);
        std::lock_guard<std::mutex> g(ctx->graph_mu);
        auto it = ctx->graphs->entries.find(key);
        if (it != ctx->graphs->entries.end()) {
            BC_HIP(hipGraphLaunch(it->second.exec, st));
            return;
        }
        // First call of this shape: run eagerly (warms the pool and the
        // coefficient tables), then record the same launch sequence.
        run_compare_split(ctx, keys, ndigits, A.data(), B.data(), lt_out, max_out, min_out, st);
        BC_HIP(hipStreamSynchronize(st));
        GraphEntry e;
        {
            std::lock_guard<std::mutex> pg(ctx->pool.mu);
            ctx->pool.recording = true;
            ctx->pool.recorded.clear();
        }
        // Record on a private stream (the legacy default stream cannot be
        // captured); the workspace lookups still use the caller's stream tag,
        // so the recording reuses the blocks of the eager run above.
        if (!ctx->capture_stream) BC_HIP(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
        hipStream_t cap = ctx->capture_stream;
        BC_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed));
        try {
            run_compare_split(ctx, keys, ndigits, A.data(), B.data(), lt_out, max_out, min_out, cap);
        } catch (...) {
            hipGraph_t dead = nullptr;
            (void)hipStreamEndCapture(cap, &dead);
            if (dead) (void)hipGraphDestroy(dead);
            std::lock_guard<std::mutex> pg(ctx->pool.mu);
            ctx->pool.recording = false;
            throw;
        }
        BC_HIP(hipStreamEndCapture(cap, &e.graph));
        BC_HIP(hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0));
        e.blocks = ctx->pool.detach_recorded();
        ctx->graphs->entries.emplace(key, std::move(e));
    });
}

int bc_set_tuning(bc_ctx *ctx, int32_t key, int64_t value) {
    return guard([&] {
        check_ctx(ctx);
        BC_REQUIRE(value >= 0, BC_ERR_ARG, "tuning value must be non-negative");
        if (key == BC_TUNE_NTT_CHUNK_BYTES) ctx->ntt_chunk_bytes = (size_t)value;
        else if (key == BC_TUNE_NTT_SINGLE_PASS) ctx->ntt_single_pass = value != 0;
        else if (key == BC_TUNE_FP64) ctx->fp64 = value != 0;
        else if (key == BC_TUNE_NTT_PARTS) ctx->ntt_parts = value != 0;
        else if (key == BC_TUNE_SPLIT_STREAMS) {
            BC_REQUIRE(value >= 1 && value <= 16, BC_ERR_ARG, "stream split must be in [1, 16]");
            std::lock_guard<std::mutex> g(ctx->split_mu);
            ctx->split = (int)value;
        }
        else if (key == BC_TUNE_POOL_LIMIT_BYTES) {
            std::lock_guard<std::mutex> g(ctx->pool.mu);
            ctx->pool.limit = (size_t)value;
        } else if (key == BC_TUNE_TEST_FAIL_ALLOC) {
            std::lock_guard<std::mutex> g(ctx->pool.mu);
            ctx->pool.fail_after = value;
        } else if (key == BC_TUNE_MFMA) {
            ctx->mfma = value != 0;
        } else if (key == BC_TUNE_RAW_HANDOFF) {
            ctx->raw_handoff = value != 0;
        } else if (key == BC_TUNE_MFMA_MODUP) {
            BC_REQUIRE(value == 0 || ctx->modup_mfma[ntt_parts_log(ctx)].w8, BC_ERR_ARG,
                       "modulus raising on the matrix cores needs fp64 primes above 2^33 and alpha 2^parts <= 32");
            ctx->mfma_modup = value != 0;
        } else if (key == BC_TUNE_PERSISTENT) {
            BC_REQUIRE(value == 0 || persist_supported(ctx), BC_ERR_ARG,
                       "persistent mode needs N = 2^13..2^15, primes below 2^50 and the default transform schedule");
            ctx->persistent = value != 0;
        } else throw Error(BC_ERR_ARG, "unknown tuning key");
    });
}

int bc_get_tuning(const bc_ctx *ctx, int32_t key, int64_t *value) {
    return guard([&] {
        check_ctx(ctx);
        BC_REQUIRE(value, BC_ERR_ARG, "null output");
        if (key == BC_TUNE_NTT_CHUNK_BYTES) *value = (int64_t)ctx->ntt_chunk_bytes;
        else if (key == BC_TUNE_NTT_SINGLE_PASS) *value = ctx->ntt_single_pass;
        else if (key == BC_TUNE_FP64) *value = ctx->fp64 && ctx->twf != nullptr;
        else if (key == BC_TUNE_NTT_PARTS) *value = ntt_parts_log(ctx);
        else if (key == BC_TUNE_SPLIT_STREAMS) *value = ctx->split;
        else if (key == BC_TUNE_POOL_LIMIT_BYTES) *value = (int64_t)ctx->pool.limit;
        else if (key == BC_TUNE_TEST_FAIL_ALLOC) *value = ctx->pool.fail_after;
        else if (key == BC_TUNE_PERSISTENT) *value = ctx->persistent;
        else if (key == BC_TUNE_MFMA) *value = ctx->mfma;
        else if (key == BC_TUNE_RAW_HANDOFF) *value = ctx->raw_handoff;
        else if (key == BC_TUNE_MFMA_MODUP) *value = ctx->mfma_modup;
        else throw Error(BC_ERR_ARG, "unknown tuning key");
    });
}

int bc_autotune(bc_ctx *ctx, void *stream) {
    return guard([&] {
        check_ctx(ctx);
        StreamScope sc(stream);
        hipStream_t st = (hipStream_t)stream;
        const int N = ctx->N, nl = ctx->nQ;
        const size_t per_poly = (size_t)nl * N * sizeof(u64);
        const int count = (int)std::max<size_t>(4, ((size_t)384 << 20) / per_poly);
        BufP buf = make_buf(ctx, per_poly * count);
        BC_HIP(hipMemsetAsync(buf->p, 0, per_poly * count, st));
        LimbSet ls{};
        ls.base = (u64 *)buf->p;
        ls.poly_stride = (u64)nl * N;
        ls.npoly = count;
        ls.nlimb = nl;
        for (int i = 0; i < nl; i++) {
            ls.off[i] = (int16_t)i;
            ls.prime[i] = (int16_t)i;
        }
        struct Cand {
            int single;
            size_t chunk;
            int fp;
        };
        std::vector<Cand> cands;
        for (int fp : {1, 0}) {
            if (fp && !ctx->twf) continue;
            cands.push_back({0, 0, fp});
            cands.push_back({0, (size_t)128 << 20, fp});
            if (ctx->logN >= 12 && ctx->logN <= 15) cands.push_back({1, 0, fp});
        }
        const bool prof = ctx->prof->on;
        ctx->prof->on = false;
        hipEvent_t e0, e1;
        BC_HIP(hipEventCreate(&e0));
        BC_HIP(hipEventCreate(&e1));
        float best = 1e30f;
        Cand pick = cands[0];
        for (const Cand &cd : cands) {
            ctx->ntt_single_pass = cd.single;
            ctx->ntt_chunk_bytes = cd.chunk;
            ctx->fp64 = cd.fp;
            ntt_forward(ctx, ls, st);
            ntt_inverse(ctx, ls, st);
            BC_HIP(hipEventRecord(e0, st));
            for (int r = 0; r < 3; r++) {
                ntt_forward(ctx, ls, st);
                ntt_inverse(ctx, ls, st);
            }
            BC_HIP(hipEventRecord(e1, st));
            BC_HIP(hipEventSynchronize(e1));
            float ms = 0;
            BC_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                pick = cd;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        ctx->ntt_single_pass = pick.single;
        ctx->ntt_chunk_bytes = pick.chunk;
        ctx->fp64 = pick.fp;
        ctx->prof->on = prof;
    });
}

int bc_autotune_mul(bc_ctx *ctx, const bc_keys *keys, void *stream) {
    return guard([&] {
        check_ctx(ctx);
        check_keys(ctx, keys);
        StreamScope sc(stream);
        hipStream_t st = (hipStream_t)stream;
        const int lv = ctx->nQ - 1;
        const size_t ctb = (size_t)2 * (lv + 1) * ctx->N * sizeof(u64);
        const int count = (int)std::min<size_t>(64, std::max<size_t>(2, ((size_t)512 << 20) / ctb));
        CtB a = alloc_ct(ctx, count, lv, 2);
        BC_HIP(hipMemsetAsync(a.data, 0, ctb * count, st));  // the kernels' time does not depend on the values
        CtB out = alloc_ct(ctx, count, out_level_mul(lv, lv), 2);
        struct Cand {
            int fp, single;
            size_t chunk;
            int parts, raw, mfma;
        };
        const bool pass1 = ctx->logN >= 12 && ctx->logN <= 15;
        std::vector<Cand> cands;
        for (int fp : {1, 0}) {
            if (fp && !ctx->twf) continue;
            for (int single : {1, 0})
                for (size_t chunk : {(size_t)0, (size_t)128 << 20}) {
                    if (single && (!pass1 || chunk)) continue;  // chunking applies to the two-pass schedule
                    for (int parts : {1, 0}) {
                        if (parts && !single) continue;
                        for (int raw : {1, 0}) {
                            if (raw && !(fp && parts)) continue;
                            for (int mfma : {0, 1}) {
                                if (mfma && !fp) continue;
                                cands.push_back({fp, single, chunk, parts, raw, mfma});
                            }
                        }
                    }
                }
        }
        const bool prof = ctx->prof->on;
        ctx->prof->on = false;
        const Cand keep{ctx->fp64, ctx->ntt_single_pass, ctx->ntt_chunk_bytes, ctx->ntt_parts, ctx->raw_handoff,
                        ctx->mfma_modup};
        auto apply = [&](const Cand &cd) {
            ctx->fp64 = cd.fp;
            ctx->ntt_single_pass = cd.single;
            ctx->ntt_chunk_bytes = cd.chunk;
            ctx->ntt_parts = cd.parts;
            ctx->raw_handoff = cd.raw;
            ctx->mfma_modup = cd.mfma;
        };
        hipEvent_t e0 = nullptr, e1 = nullptr;
        float best = 1e30f;
        Cand pick = keep;
        try {
            BC_HIP(hipEventCreate(&e0));
            BC_HIP(hipEventCreate(&e1));
            for (const Cand &cd : cands) {
                apply(cd);
                if (cd.mfma && !ctx->modup_mfma[ntt_parts_log(ctx)].w8) continue;
                mul_relin(ctx, keys, a, a, out, st);
                BC_HIP(hipEventRecord(e0, st));
                for (int r = 0; r < 3; r++) mul_relin(ctx, keys, a, a, out, st);
                BC_HIP(hipEventRecord(e1, st));
                BC_HIP(hipEventSynchronize(e1));
                float ms = 0;
                BC_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) {
                    best = ms;
                    pick = cd;
                }
            }
        } catch (...) {  // the context keeps the settings it came with
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            apply(keep);
            ctx->prof->on = prof;
            throw;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        apply(pick);
        ctx->prof->on = prof;
    });
}

int bc_profile_enable(bc_ctx *ctx, int32_t on) {
    return guard([&] {
        check_ctx(ctx);
        BC_REQUIRE(ctx->exec_mode != BC_EXEC_GRAPH || !on, BC_ERR_ARG, "profiling is not available in graph mode");
        ctx->prof->clear();
        ctx->prof->on = on != 0;
    });
}

int bc_profile_read(bc_ctx *ctx, int32_t kind, double *ms, int64_t *launches, double *bytes) {
    return guard([&] {
        check_ctx(ctx);
        BC_REQUIRE(kind >= 0 && kind < kProfKinds && ms && launches && bytes, BC_ERR_ARG, "bad profile query");
        std::lock_guard<std::mutex> g(ctx->prof->mu);
        double t = 0, by = 0;
        int64_t n = 0;
        for (auto &r : ctx->prof->recs) {
            if (r.kind != kind) continue;
            BC_HIP(hipEventSynchronize(r.b));
            float e = 0;
            BC_HIP(hipEventElapsedTime(&e, r.a, r.b));
            t += e;
            by += r.bytes;
            n++;
        }
        *ms = t;
        *launches = n;
        *bytes = by;
    });
}

int bc_compare_lt(bc_ctx *ctx, const bc_keys *keys, int32_t ndigits, const bc_ctb *a_digits, const bc_ctb *b_digits,
                  bc_ctb *out, void *stream) {
    return bc_compare_max_min(ctx, keys, ndigits, a_digits, b_digits, out, nullptr, nullptr, stream);
}

}  // extern "C"
