// persist.h -- the persistent executor: launches recorded as stages of one
// persistent kernel that drains a device work queue.
//
// While a thread has a Recorder installed, the kernel launchers of the
// comparison path (element-wise, base-conversion, key-switching, transform
// and copy kernels) append a stage -- the kernel's kind, its grid and its
// arguments -- to the recorder's current lane instead of launching.  A lane
// is an ordered stream of stages (one ring size, one context); lanes are
// independent.  The executor lays the stages of all lanes out in one ticket
// space, interleaving the lanes stage by stage and keeping each lane's order,
// and one launch of k_persist runs them: every workgroup takes the next
// ticket from a device counter, waits until the stage before it in its lane
// has finished every ticket, runs the ticket's virtual blocks through the
// same device bodies the ordinary kernels use, and counts the ticket done.
// Every dependency points to lower tickets, which running workgroups hold,
// so the queue always drains; a bounded wait flags a stall instead of
// hanging.
#pragma once

#include "bc_internal.h"

namespace bc {

// Stage kinds: one per device body (and template variant) the executor runs.
// The arithmetic is fp64 throughout (contexts whose primes are below 2^50).
enum PKind : int {
    kPkTensor = 0,
    kPkTensorAdd,
    kPkAddSub,
    kPkMulScalar,
    kPkAddConst,
    kPkLincombFp,
    kPkLincombInt,
    kPkModUp0,
    kPkModUp1,
    kPkModUp2,
    kPkKsInner,
    kPkRelinMs0,
    kPkRelinMs1,
    kPkRelinMs2,
    kPkModDown0,
    kPkModDown1,
    kPkModDown2,
    kPkKsCombine,
    kPkNttFwd0,  // whole 2^13-word limbs (N = 2^13)
    kPkNttInv0,
    kPkNttComb0,
    kPkNttFwd1,  // halves of 2^14-word limbs
    kPkNttInv1,
    kPkNttComb1,
    kPkNttFwd2,  // quarters of 2^15-word limbs
    kPkNttInv2,
    kPkNttComb2,
    kPkCopy,
    kPkKinds
};

// Arguments of each kind, as the bodies take them.
struct PaTensor {
    const u64 *a, *b, *c;
    u64 *out;
    int bcount, nl, na, nb, nc;
    const PrimeInfo *pinfo;
    int N;
};
struct PaAddSub {
    const u64 *a, *b;
    u64 *out;
    int bcount, nl, na, nb, ncomp, sub;
    const PrimeInfo *pinfo;
    int N;
};
struct PaScalar {
    const u64 *a;
    u64 *out;
    int nl, ncomp;
    ScalarArg s;
    const PrimeInfo *pinfo;
    int N;
};
struct PaLincomb {
    BabyArg ba;
    const u64 *coef;
    u64 *out;
    int nbaby, nblk, count, ct0, nl;
    const PrimeInfo *pinfo;
    int N;
};
struct PaModUp {
    const u64 *xc;
    u64 *mu;
    const ModUpPlan *plans;
    const PrimeInfo *pinfo;
    int nl, next, dnum, N;
};
struct PaKsInner {
    const u64 *mu, *x;
    size_t x_ct_stride;
    const u64 *key;
    u64 *acc;
    int level, nQ, nmod, next, nact, dnum, alpha, count;
    const PrimeInfo *pinfo;
    int N;
};
struct PaRelinMs {
    const u64 *acc, *d;
    size_t d_ct_stride;
    u64 *E;
    const ModDownPlan *md;
    const ModSwitchPlan *ms;
    const PrimeInfo *pinfo;
    int level, nQ, nP, next, N;
};
struct PaModDown {
    const u64 *acc;
    u64 *th;
    const ModDownPlan *pl;
    const PrimeInfo *pinfo;
    int level, nQ, nP, next, N;
};
struct PaKsCombine {
    const u64 *base0, *base1;
    size_t base_ct_stride;
    const u64 *acc, *th;
    u64 *out;
    size_t out_ct_stride;
    const ModDownPlan *pl;
    const PrimeInfo *pinfo;
    int nl, next, N;
};
struct PaNtt {
    LimbSet ls;
    const void *tw;
    const PrimeInfo *pinfo;
    NttCombine cb;  // combine kinds only
};
// rows x width words from src (row pitch spitch words) to dst (dpitch);
// a virtual block copies 512 words of one row
struct PaCopy {
    const u64 *src;
    u64 *dst;
    u64 spitch, dpitch, width;
};
constexpr int kCopyBlockWords = 512;

// Device descriptor of one stage (48 bytes).
struct PStage {
    int kind;
    int gx, gy, gz;  // virtual grid
    int per;         // virtual blocks per ticket
    int start;       // first ticket
    int ntick;       // tickets
    int dep;         // stage whose tickets must all be done first (-1: none)
    int args;        // byte offset of the arguments (16-byte aligned)
    int pad[3];
};

// Queues: one per XCD when the lanes are pinned to XCDs (each XCD's
// workgroups take only its tickets, and a hand-off stays inside one L2), else
// one for the device.
constexpr int kMaxXcd = 16;

// Queue state in device memory: zeroed before every launch.
struct PQueue {
    int next[kMaxXcd];  // next ticket of each queue
    int stalled;        // a bounded wait expired, or a queue was left undrained
    int exited;         // workgroups that have left
    int pad[2];
    int done[1];        // tickets done per stage (nstage entries)
};

// The queues' shape (uploaded with the plan, after the queue state).
struct PHeader {
    int nq;                // queues (1: device-wide, else one per XCD)
    int ntick[kMaxXcd];    // tickets of each queue
    int map_off[kMaxXcd];  // where each queue's ticket -> stage map starts
};

struct Recorder {
    struct S {
        PStage st;
        int lane;
        std::vector<char> args;
    };
    int lane = 0;
    std::vector<S> stages;
    // queues of the layout: 1 (device-wide), or the number of XCDs, lane l
    // then running on XCD lane_xcd[l]
    int nq = 1;
    std::vector<int> lane_xcd;
    // grid of virtual blocks; `per` = 0 picks the blocks per ticket from the
    // stage's size
    template <class T>
    void add(int kind, dim3 grid, const T &a, int per = 0) {
        S s{};
        s.st.kind = kind;
        s.st.gx = (int)grid.x;
        s.st.gy = (int)grid.y;
        s.st.gz = (int)grid.z;
        s.st.per = per;
        s.lane = lane;
        s.args.assign((const char *)&a, (const char *)&a + sizeof(T));
        if ((long long)grid.x * grid.y * grid.z > 0) stages.push_back(std::move(s));
    }
};
extern thread_local Recorder *tl_rec;

// A recording laid out for the executor: one host image of the device table
// [queue state | queue shape | stages | ticket -> stage maps | arguments].
struct PersistPlan {
    std::vector<char> image;
    size_t off_head = 0, off_stage = 0, off_map = 0, off_args = 0;
    int nstage = 0, ntick = 0, nq = 1;
};
PersistPlan persist_plan(const Recorder &rec);
// Runs an uploaded plan on `st`: the queue state is zeroed by a small kernel,
// then one persistent launch drains the queue.  stall_flag: pinned host word
// the kernel sets to 1 when a bounded wait expires (the results are then not
// valid).
void persist_run(const PersistPlan &plan, void *table, int *stall_flag, hipStream_t st);
// Workgroups of the persistent launch (resident capacity of the device).
int persist_grid();
// XCDs of the current device (1 when the runtime does not say).
int persist_xcds();
struct PersistShape {
    int stages, tickets, grid;
};

// Upload-and-launch state of one caller of the executor (a group, or a
// context's comparison calls): pinned staging for the table image (reused
// once the copy from it has run), the pinned stall flag, and the shape of the
// last launch.
struct PersistRunner {
    void *staging = nullptr;
    size_t staging_bytes = 0;
    hipEvent_t staging_free = nullptr;
    int *stall = nullptr;
    PersistShape last{};
    PersistRunner();
    ~PersistRunner();
    PersistRunner(const PersistRunner &) = delete;
    PersistRunner &operator=(const PersistRunner &) = delete;
    // BC_ERR_HIP (once) when an earlier launch of this runner stalled
    void check_stall();
    // lays out `rec`, uploads it into a workspace block of `c`'s pool on `st`
    // and launches it there
    void run(bc_ctx *c, const Recorder &rec, hipStream_t st);
};

}  // namespace bc
