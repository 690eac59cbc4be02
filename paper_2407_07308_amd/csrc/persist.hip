// persist.hip -- the persistent executor (persist.h): one launch of k_persist
// runs every recorded stage of every lane from a device work queue.
//
// The paper's answer to low GPU utilisation is to batch heterogeneous work
// (comparisons of different sizes, digits, pairs) onto the device at once
// (The Design of BoostCom, heterogeneous parallelization and GPU-related
// Optimizations).  Here ring sizes N = 2^13, 2^14, 2^15 meet in one kernel:
// every transform stage of every size is cut into 2^13-word blocks (whole
// limbs at 2^13, halves at 2^14, quarters at 2^15; the neighbouring kernels
// fold the outer stages), so one 256-thread workgroup shape with one 33 KB
// LDS buffer runs every stage kind, and the workgroups stay resident while
// tickets of all lanes flow through them.
//
// Ordering: a ticket may start once every ticket of the stage before it in
// its lane is done.  Producers make their stores visible to the whole device
// (every wave waits for its stores, then one release and one counter
// increment per ticket);
// consumers wait on the counter (one lane of one wave, bounded by a wall
// clock) and then acquire (each wave invalidates the L1 after the barrier).  A
// workgroup that runs several tickets after the same dependency acquires it
// once.

#include "kernels_dev.h"
#include "ntt_dev.h"
#include "persist.h"

#include <algorithm>

namespace bc {

thread_local Recorder *tl_rec = nullptr;

namespace {

constexpr int kPT = 256;                               // threads of every body
constexpr int kPLds = ntt_lds_words(13, 1, true);      // 2^13-word blocks, two-round exchange
static_assert(kPLds == ntt_lds_words(13, 2, true) && kPLds == ntt_lds_words(13, 0, true), "one LDS size");
constexpr unsigned long long kStallTicks = 2ull * 100000000ull;  // 2 s of the 100 MHz wall clock

__device__ __forceinline__ VBlk vblk_of(int gx, int gy, int gz, int v) {
    VBlk b;
    b.gx = gx;
    b.gy = gy;
    b.gz = gz;
    b.x = v % gx;
    const int r = v / gx;
    b.y = r % gy;
    b.z = r / gy;
    return b;
}

__device__ __forceinline__ void b_copy(const VBlk &VB, const PaCopy &a) {
    const u64 row = (u64)VB.y, x0 = (u64)VB.x * kCopyBlockWords;
    const u64 x1 = x0 + kCopyBlockWords < a.width ? x0 + kCopyBlockWords : a.width;
    const u64 *s = a.src + row * a.spitch;
    u64 *d = a.dst + row * a.dpitch;
    for (u64 k = x0 + threadIdx.x; k < x1; k += kPT) d[k] = s[k];
}


// One virtual block of each stage kind, each its own function so that every
// body gets the whole register budget (inlined into one switch, the bodies'
// live ranges pile up and spill).
#define PK_FN(name) __device__ __noinline__ void name(const char *__restrict__ A, VBlk vb, int v, u64 *lds)
PK_FN(pk_tensor) {
    const PaTensor &a = *reinterpret_cast<const PaTensor *>(A);
    b_tensor<false>(vb, a.a, a.b, a.c, a.out, a.bcount, a.nl, a.na, a.nb, a.nc, a.pinfo, a.N);
}
PK_FN(pk_tensor_add) {
    const PaTensor &a = *reinterpret_cast<const PaTensor *>(A);
    b_tensor<true>(vb, a.a, a.b, a.c, a.out, a.bcount, a.nl, a.na, a.nb, a.nc, a.pinfo, a.N);
}
PK_FN(pk_addsub) {
    const PaAddSub &a = *reinterpret_cast<const PaAddSub *>(A);
    b_addsub(vb, a.a, a.b, a.out, a.bcount, a.nl, a.na, a.nb, a.ncomp, a.sub, a.pinfo, a.N);
}
PK_FN(pk_mul_scalar) {
    const PaScalar &a = *reinterpret_cast<const PaScalar *>(A);
    b_mul_scalar(vb, a.a, a.out, a.nl, a.ncomp, a.s, a.pinfo, a.N);
}
PK_FN(pk_add_const) {
    const PaScalar &a = *reinterpret_cast<const PaScalar *>(A);
    b_add_const(vb, a.a, a.out, a.nl, a.ncomp, a.s, a.pinfo, a.N);
}
template <bool FP>
PK_FN(pk_lincomb) {
    const PaLincomb &a = *reinterpret_cast<const PaLincomb *>(A);
    b_lincomb<FP>(vb, a.ba, a.coef, a.out, a.nbaby, a.nblk, a.count, a.ct0, a.nl, a.pinfo, a.N);
}
template <int PL>
PK_FN(pk_modup) {
    const PaModUp &a = *reinterpret_cast<const PaModUp *>(A);
    b_modup<true, PL, PL ? kFoldDigit : kMaxDigit>(vb, a.xc, a.mu, a.plans, a.pinfo, a.nl, a.next, a.dnum, a.N);
}
PK_FN(pk_ks_inner) {
    const PaKsInner &a = *reinterpret_cast<const PaKsInner *>(A);
    b_ks_inner<true>(vb, a.mu, a.x, a.x_ct_stride, a.key, a.acc, a.level, a.nQ, a.nmod, a.next, a.nact, a.dnum,
                     a.alpha, a.count, a.pinfo, a.N);
}
template <int PL>
PK_FN(pk_relin_ms) {
    const PaRelinMs &a = *reinterpret_cast<const PaRelinMs *>(A);
    b_relin_ms_fbc<true, PL, PL ? kFoldDigit : kMaxDigit>(vb, a.acc, a.d, a.d_ct_stride, a.E, a.md, a.ms, a.pinfo,
                                                          a.level, a.nQ, a.nP, a.next, a.N);
}
template <int PL>
PK_FN(pk_moddown) {
    const PaModDown &a = *reinterpret_cast<const PaModDown *>(A);
    b_moddown<true, PL>(vb, a.acc, a.th, a.pl, a.pinfo, a.level, a.nQ, a.nP, a.next, a.N);
}
PK_FN(pk_ks_combine) {
    const PaKsCombine &a = *reinterpret_cast<const PaKsCombine *>(A);
    b_ks_combine(vb, a.base0, a.base1, a.base_ct_stride, a.acc, a.th, a.out, a.out_ct_stride, a.pl, a.pinfo, a.nl,
                 a.next, a.N);
}
template <int PL, bool INV, int EPI>
PK_FN(pk_ntt) {
    const PaNtt &a = *reinterpret_cast<const PaNtt *>(A);
    ntt_full_body<13, INV, FpA, EPI, PL, true>(a.ls, a.tw, a.pinfo, &a.cb, v, lds);
}
PK_FN(pk_copy) { b_copy(vb, *reinterpret_cast<const PaCopy *>(A)); }
#undef PK_FN

__device__ __forceinline__ void run_block(int kind, const char *__restrict__ A, const VBlk &vb, int v, u64 *lds) {
    switch (kind) {
        case kPkTensor: pk_tensor(A, vb, v, lds); break;
        case kPkTensorAdd: pk_tensor_add(A, vb, v, lds); break;
        case kPkAddSub: pk_addsub(A, vb, v, lds); break;
        case kPkMulScalar: pk_mul_scalar(A, vb, v, lds); break;
        case kPkAddConst: pk_add_const(A, vb, v, lds); break;
        case kPkLincombFp: pk_lincomb<true>(A, vb, v, lds); break;
        case kPkLincombInt: pk_lincomb<false>(A, vb, v, lds); break;
        case kPkModUp0: pk_modup<0>(A, vb, v, lds); break;
        case kPkModUp1: pk_modup<1>(A, vb, v, lds); break;
        case kPkModUp2: pk_modup<2>(A, vb, v, lds); break;
        case kPkKsInner: pk_ks_inner(A, vb, v, lds); break;
        case kPkRelinMs0: pk_relin_ms<0>(A, vb, v, lds); break;
        case kPkRelinMs1: pk_relin_ms<1>(A, vb, v, lds); break;
        case kPkRelinMs2: pk_relin_ms<2>(A, vb, v, lds); break;
        case kPkModDown0: pk_moddown<0>(A, vb, v, lds); break;
        case kPkModDown1: pk_moddown<1>(A, vb, v, lds); break;
        case kPkModDown2: pk_moddown<2>(A, vb, v, lds); break;
        case kPkKsCombine: pk_ks_combine(A, vb, v, lds); break;
        case kPkNttFwd0: pk_ntt<0, false, 0>(A, vb, v, lds); break;
        case kPkNttInv0: pk_ntt<0, true, 0>(A, vb, v, lds); break;
        case kPkNttComb0: pk_ntt<0, false, kNttRelinMs>(A, vb, v, lds); break;
        case kPkNttFwd1: pk_ntt<1, false, 0>(A, vb, v, lds); break;
        case kPkNttInv1: pk_ntt<1, true, 0>(A, vb, v, lds); break;
        case kPkNttComb1: pk_ntt<1, false, kNttRelinMs>(A, vb, v, lds); break;
        case kPkNttFwd2: pk_ntt<2, false, 0>(A, vb, v, lds); break;
        case kPkNttInv2: pk_ntt<2, true, 0>(A, vb, v, lds); break;
        case kPkNttComb2: pk_ntt<2, false, kNttRelinMs>(A, vb, v, lds); break;
        case kPkCopy: pk_copy(A, vb, v, lds); break;
        default: break;
    }
}

__device__ __forceinline__ bool uses_lds(int kind) { return kind >= kPkNttFwd0 && kind <= kPkNttComb2; }

// Every workgroup: take a ticket of its queue, wait for its lane's previous
// stage, run its virtual blocks, count it done; until the tickets run out.
// The next ticket is taken while the current one runs (the queue still
// drains: the lowest unfinished ticket is always the one its holder runs
// next).  With one queue per XCD a workgroup serves its own XCD's queue,
// whose lanes never depend on another XCD: a hand-off then needs the
// producer's stores in the shared L2 (each wave waits for its stores) and the
// consumer's L1 invalidated, and no L2 is written back or invalidated.  With
// one device-wide queue the hand-off releases and acquires at agent scope.
__global__ void __launch_bounds__(kPT, 3) k_persist(const PStage *__restrict__ stages, const int *__restrict__ tmap,
                                                    const char *__restrict__ args, PQueue *q,
                                                    const PHeader *__restrict__ hd, int *stall_flag) {
    __shared__ u64 lds[kPLds];
    __shared__ int sh_next;
    const int nq = __builtin_amdgcn_readfirstlane(hd->nq);
    const bool local = nq > 1;
    // this workgroup's XCD (hardware register XCC_ID, 4 bits)
    const int x = local ? (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) % (unsigned)nq) : 0;
    const int ntick = __builtin_amdgcn_readfirstlane(hd->ntick[x]);
    const int *map = tmap + __builtin_amdgcn_readfirstlane(hd->map_off[x]);
    if (threadIdx.x == 0) sh_next = __hip_atomic_fetch_add(&q->next[x], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    int acquired = -1;  // the dependency this workgroup has acquired last
    for (;;) {
        const int t = __builtin_amdgcn_readfirstlane(sh_next);
        __syncthreads();  // every wave has read sh_next
        if (t >= ntick) break;
        if (threadIdx.x == 0)
            sh_next = __hip_atomic_fetch_add(&q->next[x], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int si = __builtin_amdgcn_readfirstlane(map[t]);
        const PStage &S = stages[si];
        const int dep = __builtin_amdgcn_readfirstlane(S.dep);
        if (dep >= 0 && dep != acquired) {
            if (threadIdx.x == 0) {
                const int target = stages[dep].ntick;
                const unsigned long long t0 = wall_clock64();
                while (__hip_atomic_load(&q->done[dep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                    __builtin_amdgcn_s_sleep(4);
                    // one expired wait ends every other wait at once
                    if (__hip_atomic_load(&q->stalled, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                    if (wall_clock64() - t0 > kStallTicks) {
                        __hip_atomic_store(&q->stalled, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_store(stall_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                        break;
                    }
                }
            }
            __syncthreads();
            // every wave acquires for itself after the barrier (the barrier
            // does not order one wave's cache invalidation before another
            // wave's loads): the L1 alone when the producer shares this XCD's
            // L2, else the agent-scope acquire
            if (local) asm volatile("buffer_inv sc0\n\ts_waitcnt vmcnt(0)" ::: "memory");
            else __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            acquired = dep;
        }
        const int kind = __builtin_amdgcn_readfirstlane(S.kind);
        const int gx = __builtin_amdgcn_readfirstlane(S.gx), gy = __builtin_amdgcn_readfirstlane(S.gy),
                  gz = __builtin_amdgcn_readfirstlane(S.gz), per = __builtin_amdgcn_readfirstlane(S.per);
        const int nvb = gx * gy * gz;
        const int v0 = (t - __builtin_amdgcn_readfirstlane(S.start)) * per;
        const int v1 = v0 + per < nvb ? v0 + per : nvb;
        const char *A = args + __builtin_amdgcn_readfirstlane(S.args);
        for (int v = v0; v < v1; v++) {
            run_block(kind, A, vblk_of(gx, gy, gz, v), v, lds);
            if (uses_lds(kind)) __syncthreads();  // the next block reuses the exchange buffer
        }
        // every wave's stores have reached the XCD's L2; then (device-wide
        // queue) one write-back of that L2 before the ticket counts
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) {
            if (!local) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(&q->done[si], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    // the last workgroup out checks that every queue was drained (a queue of
    // an XCD that received no workgroup would not be: reported as a stall)
    if (threadIdx.x == 0 &&
        __hip_atomic_fetch_add(&q->exited, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (int)gridDim.x - 1) {
        for (int y = 0; y < nq; y++)
            if (__hip_atomic_load(&q->next[y], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < hd->ntick[y]) {
                __hip_atomic_store(&q->stalled, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(stall_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
    }
}

__global__ void k_persist_reset(PQueue *q, int nstage) {
    if (threadIdx.x < kMaxXcd) q->next[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        q->stalled = 0;
        q->exited = 0;
    }
    for (int i = threadIdx.x; i < nstage; i += blockDim.x) q->done[i] = 0;
}

}  // namespace

int persist_grid() {
    static std::mutex mu;
    static int cached[64] = {0};
    int dev = 0;
    BC_HIP(hipGetDevice(&dev));
    BC_REQUIRE(dev >= 0 && dev < 64, BC_ERR_HIP, "device index out of range");
    std::lock_guard<std::mutex> g(mu);
    if (!cached[dev]) {
        int per_cu = 0, cus = 0;
        BC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persist, kPT, 0));
        BC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        BC_REQUIRE(per_cu >= 1 && cus >= 1, BC_ERR_HIP, "persistent executor: no resident workgroup fits");
        cached[dev] = per_cu * cus;
    }
    return cached[dev];
}

int persist_xcds() {
    static std::mutex mu;
    static int cached[64] = {0};
    int dev = 0;
    BC_HIP(hipGetDevice(&dev));
    BC_REQUIRE(dev >= 0 && dev < 64, BC_ERR_HIP, "device index out of range");
    std::lock_guard<std::mutex> g(mu);
    if (!cached[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess) {
            (void)hipGetLastError();
            n = 1;
        }
        cached[dev] = std::max(1, std::min(n, kMaxXcd));
    }
    return cached[dev];
}

PersistPlan persist_plan(const Recorder &rec) {
    PersistPlan p;
    const int nq = std::max(1, std::min(rec.nq, kMaxXcd));
    p.nq = nq;
    // lanes in order of first appearance; stages of a lane in recording order
    std::vector<int> lane_ids;
    std::vector<std::vector<int>> lanes;
    for (int i = 0; i < (int)rec.stages.size(); i++) {
        const int l = rec.stages[i].lane;
        auto it = std::find(lane_ids.begin(), lane_ids.end(), l);
        if (it == lane_ids.end()) {
            lane_ids.push_back(l);
            lanes.emplace_back();
            it = lane_ids.end() - 1;
        }
        lanes[it - lane_ids.begin()].push_back(i);
    }
    auto queue_of = [&](int lane) {
        if (nq == 1) return 0;
        BC_REQUIRE(lane >= 0 && lane < (int)rec.lane_xcd.size(), BC_ERR_ARG, "persistent executor: lane without XCD");
        return rec.lane_xcd[lane] % nq;
    };
    // per queue: its lanes interleaved stage by stage, each lane in order
    std::vector<int> order, dep, qof;
    std::vector<int> last(lanes.size(), -1);
    size_t depth = 0;
    for (auto &l : lanes) depth = std::max(depth, l.size());
    for (int x = 0; x < nq; x++)
        for (size_t r = 0; r < depth; r++)
            for (size_t l = 0; l < lanes.size(); l++)
                if (r < lanes[l].size() && queue_of(lane_ids[l]) == x) {
                    dep.push_back(last[l]);
                    last[l] = (int)order.size();
                    order.push_back(lanes[l][r]);
                    qof.push_back(x);
                }
    // resident workgroups serving one queue
    const int grid = std::max(1, persist_grid() / nq);
    std::vector<PStage> st(order.size());
    std::vector<char> args;
    PHeader hd{};
    hd.nq = nq;
    int ntick = 0;
    for (size_t k = 0; k < order.size(); k++) {
        const Recorder::S &s = rec.stages[order[k]];
        const int x = qof[k];
        PStage &d = st[k];
        d = s.st;
        const long long nvb = (long long)d.gx * d.gy * d.gz;
        BC_REQUIRE(nvb > 0 && nvb < (1ll << 30), BC_ERR_ARG, "persistent executor: stage grid out of range");
        // a stage's tickets: at most one per workgroup of its queue (few and
        // large: every ticket ends with a hand-off)
        if (d.per <= 0) d.per = (int)std::max<long long>(1, (nvb + grid - 1) / grid);
        d.ntick = (int)((nvb + d.per - 1) / d.per);
        d.start = hd.ntick[x];  // tickets are numbered inside the queue
        d.dep = dep[k];
        BC_REQUIRE(d.dep < (int)k && (d.dep < 0 || qof[d.dep] == x), BC_ERR_ARG,
                   "persistent executor: dependency order");
        hd.ntick[x] += d.ntick;
        ntick += d.ntick;
        BC_REQUIRE(ntick < (1 << 30), BC_ERR_ARG, "persistent executor: too many tickets");
        args.resize((args.size() + 15) / 16 * 16);
        d.args = (int)args.size();
        args.insert(args.end(), s.args.begin(), s.args.end());
        BC_REQUIRE(args.size() < (1u << 31), BC_ERR_ARG, "persistent executor: arguments too large");
    }
    for (int x = 1; x < nq; x++) hd.map_off[x] = hd.map_off[x - 1] + hd.ntick[x - 1];
    p.nstage = (int)st.size();
    p.ntick = ntick;
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    p.off_head = up(offsetof(PQueue, done) + sizeof(int) * std::max(1, p.nstage));
    p.off_stage = up(p.off_head + sizeof(PHeader));
    p.off_map = up(p.off_stage + sizeof(PStage) * st.size());
    p.off_args = up(p.off_map + sizeof(int) * (size_t)ntick);
    p.image.assign(up(p.off_args + args.size()), 0);
    std::memcpy(p.image.data() + p.off_head, &hd, sizeof hd);
    if (!st.empty()) std::memcpy(p.image.data() + p.off_stage, st.data(), sizeof(PStage) * st.size());
    int *map = reinterpret_cast<int *>(p.image.data() + p.off_map);
    for (size_t k = 0; k < st.size(); k++)
        for (int t = 0; t < st[k].ntick; t++) map[hd.map_off[qof[k]] + st[k].start + t] = (int)k;
    if (!args.empty()) std::memcpy(p.image.data() + p.off_args, args.data(), args.size());
    return p;
}

PersistRunner::PersistRunner() {
    BC_HIP(hipEventCreateWithFlags(&staging_free, hipEventDisableTiming));
    BC_HIP(hipHostMalloc((void **)&stall, sizeof(int), hipHostMallocDefault));
    *stall = 0;
}

PersistRunner::~PersistRunner() {
    if (staging) (void)hipHostFree(staging);
    if (stall) (void)hipHostFree(stall);
    if (staging_free) (void)hipEventDestroy(staging_free);
}

void PersistRunner::check_stall() {
    if (*(volatile int *)stall) {
        *stall = 0;
        throw Error(BC_ERR_HIP, "an earlier persistent launch stalled: the results of that call are invalid");
    }
}

void PersistRunner::run(bc_ctx *c, const Recorder &rec, hipStream_t st) {
    const PersistPlan plan = persist_plan(rec);
    last = PersistShape{plan.nstage, plan.ntick, persist_grid()};
    if (plan.ntick == 0) return;
    // the table is a workspace block tagged with the launch stream, handed back
    // once the launch is queued (stream order protects its reuse)
    struct Block {
        Pool &pool;
        void *ptr = nullptr;
        ~Block() { pool.release(ptr); }
    } blk{c->pool};
    hipStream_t prev = tl_stream;
    tl_stream = st;
    try {
        blk.ptr = c->pool.alloc(plan.image.size());
        void *table = blk.ptr;
        BC_HIP(hipEventSynchronize(staging_free));  // the last upload has read the staging buffer
        if (staging_bytes < plan.image.size()) {
            if (staging) BC_HIP(hipHostFree(staging));
            staging = nullptr;
            staging_bytes = 0;
            BC_HIP(hipHostMalloc(&staging, plan.image.size(), hipHostMallocDefault));
            staging_bytes = plan.image.size();
        }
        std::memcpy(staging, plan.image.data(), plan.image.size());
        BC_HIP(hipMemcpyAsync(table, staging, plan.image.size(), hipMemcpyHostToDevice, st));
        BC_HIP(hipEventRecord(staging_free, st));
        persist_run(plan, table, stall, st);
    } catch (...) {
        tl_stream = prev;
        throw;
    }
    tl_stream = prev;
}

void persist_run(const PersistPlan &plan, void *table, int *stall_flag, hipStream_t st) {
    if (plan.ntick == 0) return;
    char *base = (char *)table;
    PQueue *q = reinterpret_cast<PQueue *>(base);
    k_persist_reset<<<1, kPT, 0, st>>>(q, plan.nstage);
    k_persist<<<persist_grid(), kPT, 0, st>>>(reinterpret_cast<const PStage *>(base + plan.off_stage),
                                             reinterpret_cast<const int *>(base + plan.off_map), base + plan.off_args,
                                             q, reinterpret_cast<const PHeader *>(base + plan.off_head), stall_flag);
    BC_HIP(hipGetLastError());
}

}  // namespace bc
