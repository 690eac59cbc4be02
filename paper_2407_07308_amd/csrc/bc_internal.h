// bc_internal.h -- shared declarations of the gfx950 BGV library (device
// arithmetic, context layout, launch descriptors).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/boostcom.h"

namespace bc {

typedef uint64_t u64;
typedef uint32_t u32;
typedef int64_t i64;
typedef unsigned __int128 u128;

constexpr int kMaxMod = 40;    // nQ + nP
constexpr int kMaxJobs = 160;  // limbs listed in one transform launch
constexpr int kMaxDigit = 16;  // primes per key-switching digit, and special primes
constexpr int kFoldDigit = 8;  // the same bound for the kernels that fold transform stages
constexpr int kWideMfmaK = 128, kWideMfmaM = 256;  // largest outputs / inputs of the matrix-core combination

// ------------------------------------------------------------------ errors

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define BC_HIP(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            throw ::bc::Error(BC_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));     \
    } while (0)

#define BC_REQUIRE(cond, code, msg)                                                               \
    do {                                                                                          \
        if (!(cond)) throw ::bc::Error((code), (msg));                                            \
    } while (0)

// ------------------------------------------------------- device arithmetic
// Residues are below q < 2^61.  Lazy values stay below 4q < 2^63.

__device__ __forceinline__ u64 mulhi(u64 a, u64 b) { return __umul64hi(a, b); }

// Shoup multiplication by a constant w < q with wp = floor(w 2^64 / q):
// a w - floor(a wp / 2^64) q lies in [0, 2q) for every a < 2^64.
__device__ __forceinline__ u64 shoup_lazy(u64 a, u64 w, u64 wp, u64 q) { return a * w - mulhi(a, wp) * q; }

__device__ __forceinline__ u64 shoup(u64 a, u64 w, u64 wp, u64 q) {
    u64 r = shoup_lazy(a, w, wp, q);
    return r >= q ? r - q : r;
}

__device__ __forceinline__ u64 add_mod(u64 a, u64 b, u64 q) {
    u64 s = a + b;
    return s >= q ? s - q : s;
}

__device__ __forceinline__ u64 sub_mod(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + q - b; }

// ------------------------------------------- exact fp64 residue arithmetic
// For primes below 2^50 a residue can be held as an integer-valued double and
// multiplied at the full fp64 rate.  A constant w (0 <= w < q) travels as the
// pair (w, w/q) of doubles (FPair; stored in the two words of a Shoup pair).
// f_mulmod(y, c) for |y| < 2^52: quotient estimate k = rint(y * (w/q)), off
// from y w / q by at most 1/2 + |y| 2^-52; the exact split y w = ph + pl
// (ph = fl(y w), pl = fma(y, w, -ph)); result (ph - k q) + pl, where fma
// forms ph - k q exactly because it is an integer below 2^53 and the final
// sum is exact for the same reason.  The result is congruent to y w and
// |result| <= q (1/2 + |y| 2^-52).  f_reduce(x) = x - rint(x/q) q is exact and
// lies in [-q/2, q/2] up to one unit for |x| < 2^53.
struct FPair {
    double w, wq;
};
__device__ __forceinline__ FPair fpair(const u64 *p) {
    return {__longlong_as_double((long long)p[0]), __longlong_as_double((long long)p[1])};
}
__device__ __forceinline__ double f_mulmod(double y, FPair c, double q) {
#pragma clang fp contract(off)
    double k = __builtin_rint(y * c.wq), ph = y * c.w, pl = __builtin_fma(y, c.w, -ph);
    return __builtin_fma(-k, q, ph) + pl;
}
__device__ __forceinline__ double f_reduce(double x, double q, double qinv) {
#pragma clang fp contract(off)
    return __builtin_fma(-__builtin_rint(x * qinv), q, x);
}
// canonical representative in [0, q)
__device__ __forceinline__ double f_canon(double x, double q, double qinv) {
#pragma clang fp contract(off)
    double r = f_reduce(x, q, qinv);
    return r < 0.0 ? r + q : r;
}
// centred representative in [-(q-1)/2, (q-1)/2] (q odd)
__device__ __forceinline__ double f_centre(double x, double q, double qinv) {
#pragma clang fp contract(off)
    double r = f_reduce(x, q, qinv), h = 0.5 * (q - 1.0);
    r = r > h ? r - q : r;
    return r < -h ? r + q : r;
}
// an integer-valued double passed between kernels as its bit pattern
__device__ __forceinline__ double f_raw_load(u64 x) { return __longlong_as_double((long long)x); }
__device__ __forceinline__ u64 f_raw_bits(double x) { return (u64)__double_as_longlong(x); }
// 0 <= x < 2^52 as a double: OR-ing 2^52's exponent into the pattern gives 2^52 + x
__device__ __forceinline__ double f_load(u64 x) {
#pragma clang fp contract(off)
    return __longlong_as_double((long long)(x | 0x4330000000000000ull)) - 0x1p52;
}
// integer-valued double in [0, 2^52) -> u64
__device__ __forceinline__ u64 f_bits(double x) {
#pragma clang fp contract(off)
    return (u64)__double_as_longlong(x + 0x1p52) & 0x000FFFFFFFFFFFFFull;
}

// Per-prime Barrett data for products of two variables a, b < q:
// x = a b < q^2 < 2^(2s) (q < 2^s);  t = x >> (s-2);  qh = mulhi(t, mu),
// mu = floor(2^(62+s) / q);  then qh is floor(x/q) minus at most 2 and
// x - qh q < 3q.
struct Barrett {
    u64 q, mu;
    int sh;  // s - 2
    int pad;
};

__device__ __forceinline__ u64 mul_mod(u64 a, u64 b, const Barrett &m) {
    u64 lo = a * b, hi = mulhi(a, b);
    u64 t = (hi << (64 - m.sh)) | (lo >> m.sh);
    u64 r = lo - mulhi(t, m.mu) * m.q;
    r = r >= 2 * m.q ? r - 2 * m.q : r;
    return r >= m.q ? r - m.q : r;
}

// ------------------------------------------------------ launch descriptors

// Block coordinates a kernel body works on: the hardware's when the body runs
// as its own kernel, a virtual block's when the persistent executor runs it.
struct VBlk {
    int x, y, z;     // block index
    int gx, gy, gz;  // grid size
};
__device__ __forceinline__ VBlk hw_blk() {
    return {(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z, (int)gridDim.x, (int)gridDim.y, (int)gridDim.z};
}

// A list of residue polynomials (limbs) inside a batch: limb k of poly b sits
// at base + b * poly_stride + off[k] * N and is reduced mod prime[k].
struct LimbSet {
    u64 *base;
    u64 poly_stride;
    int npoly;
    int nlimb;
    int16_t off[kMaxJobs];
    int16_t prime[kMaxJobs];
    // out-of-place input (null: in place): limb k of poly j is read from
    // ibase + j * ipoly_stride + ioff[k] * N and written to base + ...
    const u64 *ibase;
    u64 ipoly_stride;
    int16_t ioff[kMaxJobs];
    // part-limb transforms with fp64 arithmetic: the limbs are read / written
    // as the bit patterns of reduced integer-valued doubles (|x| <= q/2)
    // instead of canonical words (between key-switching kernels only)
    int8_t raw_in = 0, raw_out = 0;
};

// A scalar's residues mod each q_i (Shoup pairs): scalar multiplication and
// constant addition.
struct ScalarArg {
    u64 w[kMaxMod][2];
};

// Paterson-Stockmeyer blocks: H[pos(t)][ct] = sum_k coef[t][k] * baby_k[ct]
// (NTT domain, every baby at the same level).  Integer kernel: coef holds
// Shoup pairs [nblk][nbaby][nl][2] of the centred coefficients mod q_i.
// fp64 kernel: coef holds the centred coefficients themselves as doubles
// [nblk][nbaby] (|c| < p/2 < 2^19): each baby word v < 2^50 is split as
// v = h 2^25 + l, the sums of c h and of c l stay below 16 2^19 2^25 = 2^48
// (exact in fp64 fused multiply-adds), and the result is
// (sum c h) (2^25 mod q) + sum c l reduced once.
struct BabyArg {
    const u64 *baby[16];
    int nlb[16];  // limbs per component each baby is stored with (>= nl: its lowest nl are read)
    int pos[64];  // storage position of block t
};

// Constants of one prime (device copy).
struct PrimeInfo {
    u64 q;
    Barrett br;
    u64 ninv, ninvp;      // N^-1 (Shoup)
    u64 ninvw1, ninvw1p;  // N^-1 * Winv[1] (Shoup): last inverse stage
    u64 p_mod, p_modp;    // p mod q (Shoup)
    // fp64 transform arithmetic (q < 2^50): q, 1/q, and N^-1, N^-1 * Winv[1]
    // each with its ratio to q
    double qd, qinv, ninv_d, ninv_q, ninvw1_d, ninvw1_q;
    u64 p_f[2];      // p mod q as an FPair (fp64 base conversions)
    u64 two25_f[2];  // 2^25 mod q as an FPair (small-coefficient linear combinations)
    // forward twiddles W[1], W[2], W[3] of the first two stages, folded into
    // the kernels that produce words for a part-limb transform: Shoup pairs
    // and FPairs
    u64 w123[3][2];
    u64 w123_f[3][2];
    // inverse twiddles Winv[2], Winv[3] of the second-to-last inverse stage
    // (N = 2^15), unfolded by the kernels that consume a part-limb inverse
    // transform: Shoup pairs and FPairs
    u64 wi23[2][2];
    u64 wi23_f[2][2];
};

// The first PL forward stages (PL = 1, 2) of a limb's transform applied to
// the 2^PL words v[j] = a[x + j N / 2^PL] of one position x: the stage of
// span N/2 pairs (v0, v1) (PL = 1) or (v0, v2), (v1, v3) with twiddle W[1],
// the stage of span N/4 pairs (v0, v1) with W[2] and (v2, v3) with W[3].
// Canonical words in and out.  What remains of the transform splits into
// 2^PL independent parts.
__device__ __forceinline__ void bfly_int(u64 &x, u64 &y, const u64 *w, u64 q) {
    const u64 p = shoup(y, w[0], w[1], q);
    y = sub_mod(x, p, q);
    x = add_mod(x, p, q);
}
template <int PL>
__device__ __forceinline__ void fold_int(u64 *v, const PrimeInfo &pi) {
    static_assert(PL == 1 || PL == 2, "one or two stages");
    if constexpr (PL == 1) {
        bfly_int(v[0], v[1], pi.w123[0], pi.q);
    } else {
        bfly_int(v[0], v[2], pi.w123[0], pi.q);
        bfly_int(v[1], v[3], pi.w123[0], pi.q);
        bfly_int(v[0], v[1], pi.w123[1], pi.q);
        bfly_int(v[2], v[3], pi.w123[2], pi.q);
    }
}
// fp64: |x|, |y| < 1.6 q in, |x| < 2.6 q out (f_mulmod's bound), exact
__device__ __forceinline__ void bfly_fp(double &x, double &y, const u64 *w, double q) {
#pragma clang fp contract(off)
    const double p = f_mulmod(y, fpair(w), q);
    y = x - p;
    x = x + p;
}
// CANON: canonical results, else reduced ones (|x| <= q/2, for consumers
// that take the fp64 pattern of the words)
template <int PL, bool CANON = true>
__device__ __forceinline__ void fold_fp(double *v, const PrimeInfo &pi) {
    static_assert(PL == 1 || PL == 2, "one or two stages");
    if constexpr (PL == 1) {
        bfly_fp(v[0], v[1], pi.w123_f[0], pi.qd);
    } else {
        bfly_fp(v[0], v[2], pi.w123_f[0], pi.qd);
        bfly_fp(v[1], v[3], pi.w123_f[0], pi.qd);
        bfly_fp(v[0], v[1], pi.w123_f[1], pi.qd);
        bfly_fp(v[2], v[3], pi.w123_f[2], pi.qd);
    }
#pragma unroll
    for (int j = 0; j < (1 << PL); j++) v[j] = CANON ? f_canon(v[j], pi.qd, pi.qinv) : f_reduce(v[j], pi.qd, pi.qinv);
}

// The last PL inverse stages (PL = 1, 2), N^-1 included, on the 2^PL words
// v[j] = a[x + j N / 2^PL] of one position after a part-limb inverse
// transform: with PL = 2 the stage of span N/4 pairs (v0, v1) with Winv[2]
// and (v2, v3) with Winv[3]; the final stage of span N/2 pairs (v0, v2),
// (v1, v3) (PL = 2) or (v0, v1) (PL = 1), scaled by N^-1 and N^-1 Winv[1].
// Canonical words in and out.
template <int PL>
__device__ __forceinline__ void unfold_int(u64 *v, const PrimeInfo &pi) {
    static_assert(PL == 1 || PL == 2, "one or two stages");
    const u64 q = pi.q;
    auto gs = [q](u64 &x, u64 &y, u64 w, u64 wp) {
        const u64 s = add_mod(x, y, q), d = sub_mod(x, y, q);
        x = s;
        y = shoup(d, w, wp, q);
    };
    auto last = [q, &pi](u64 &x, u64 &y) {
        const u64 s = add_mod(x, y, q), d = sub_mod(x, y, q);
        x = shoup(s, pi.ninv, pi.ninvp, q);
        y = shoup(d, pi.ninvw1, pi.ninvw1p, q);
    };
    if constexpr (PL == 1) {
        last(v[0], v[1]);
    } else {
        gs(v[0], v[1], pi.wi23[0][0], pi.wi23[0][1]);
        gs(v[2], v[3], pi.wi23[1][0], pi.wi23[1][1]);
        last(v[0], v[2]);
        last(v[1], v[3]);
    }
}
// fp64: sums below 4 q before the last products (f_mulmod's bound), exact;
// results below 1.5 q in magnitude, canonical only with CANON (a consumer
// that only multiplies or adds them before reducing can skip that)
template <int PL, bool CANON = true>
__device__ __forceinline__ void unfold_fp(double *v, const PrimeInfo &pi) {
#pragma clang fp contract(off)
    static_assert(PL == 1 || PL == 2, "one or two stages");
    const double q = pi.qd;
    auto last = [q, &pi](double &x, double &y) {
        const double s = x + y, d = x - y;
        x = f_mulmod(s, FPair{pi.ninv_d, pi.ninv_q}, q);
        y = f_mulmod(d, FPair{pi.ninvw1_d, pi.ninvw1_q}, q);
    };
    if constexpr (PL == 1) {
        last(v[0], v[1]);
    } else {
        const double d0 = v[0] - v[1], d1 = v[2] - v[3];
        v[0] = v[0] + v[1];
        v[2] = v[2] + v[3];
        v[1] = f_mulmod(d0, fpair(pi.wi23_f[0]), q);
        v[3] = f_mulmod(d1, fpair(pi.wi23_f[1]), q);
        last(v[0], v[2]);
        last(v[1], v[3]);
    }
    if constexpr (CANON) {
#pragma unroll
        for (int j = 0; j < (1 << PL); j++) v[j] = f_canon(v[j], q, pi.qinv);
    }
}

// Fast base conversion from one digit at one level (modulus raising).
struct ModUpPlan {
    int src_lo, nsrc;    // source primes [src_lo, src_lo + nsrc)
    int ntgt;            // target limbs (extended index e, prime index)
    int tgt_e[kMaxMod];
    int tgt_prime[kMaxMod];
    u64 qhinv[kMaxMod][2];          // [Qhat_i^-1]_{q_i}, Shoup
    u64 qhat[kMaxMod][kMaxMod][2];  // [t][i]: Qhat_i mod q_t, Shoup
};

// Split-int8 matrix-core form of modulus raising with PL folded forward
// stages: per plan (level x digit) a block of plan_stride bytes of tiles of
// 32 rows x kpad signed digits, and per (plan, target, output word) the fp64
// correction of the byte shift (see b_modup_mfma).
struct ModUpMfma {
    int8_t *w8 = nullptr;
    double *corr = nullptr;
    int kpad = 0, plan_stride = 0;
};

// Exact division by P (modulus lowering); independent of the level.
struct ModDownPlan {
    u64 vfac[kMaxMod][2];           // [p^-1 Phat_j^-1]_{p_j}
    u64 phat[kMaxMod][kMaxMod][2];  // [i][j]: Phat_j mod q_i
    u64 pinv[kMaxMod][2];           // P^-1 mod q_i
    u64 ppinv[kMaxMod][2];          // p P^-1 mod q_i
    u64 phatpp[kMaxMod][kMaxMod][2];  // [i][j]: Phat_j p P^-1 mod q_i (the scaled correction)
};

// Dropping q_l (modulus switching at level l).
struct ModSwitchPlan {
    u64 pinv_l[2];         // p^-1 mod q_l
    u64 ql;                // q_l
    u64 qlinv[kMaxMod][2]; // q_l^-1 mod q_i
    // relinearisation fused with this switch, folded constants mod q_i:
    // Phat_j p P^-1 q_l^-1 and p q_l^-1
    u64 rk1[kMaxMod][kMaxDigit][2];
    u64 rk2[kMaxMod][2];
};

// Mixed-radix (Garner) reconstruction tables for decryption.
struct GarnerTable {
    u64 inv[kMaxMod][kMaxMod][2];  // [i][j], j < i: q_j^-1 mod q_i (Shoup)
    u64 one_p[kMaxMod];            // floor(2^64 / q_i): Shoup reduction by 1
    u64 mprod_p[kMaxMod];          // prod_{j < i} q_j mod p
    u64 qprod_p[kMaxMod];          // prod_{j <= i} q_j mod p
};

// Final step of a multiplication or of a modulus switch, applied by the
// forward transform of a correction E ([count][2][level][N], coefficient
// domain in, transformed) as it stores, limbs i < level of both components:
//   kNttRelinMs:  out_i = d_i w0_i + acc_i w1_i - E_i   (relinearise + switch:
//                 w0 = q_l^-1, w1 = P^-1 q_l^-1, acc the key-switch accumulator)
//   kNttSwitch:   out_i = (d_i - E_i) w0_i               (switch: w0 = q_l^-1)
// d has level + 1 limbs per component (stride d_ct_stride per ciphertext);
// acc is [count][2][next][N].  w[i] holds the constants mod q_i as pairs of
// the transform's arithmetic (Shoup pairs, or (w, w/q) doubles).
//   kNttKsCombine: out_i = d_i w0_i + acc_i w1_i - E_i (a key switch: d the
//                 base of component 0, d1 that of component 1 (a table of N
//                 zero words, d1_limb = d1_ct_stride = 0, when it has none);
//                 w0 = 1, w1 = P^-1, E the modulus-lowering correction
//                 already scaled by p P^-1); here `level` counts the limbs of
//                 a component of E, d and out alike.
enum { kNttRelinMs = 1, kNttSwitch = 2, kNttKsCombine = 3 };
struct NttCombine {
    int mode;
    const u64 *d;
    u64 d_ct_stride;
    const u64 *acc;
    u64 *out;
    int level, next;
    u64 w[kMaxMod][4];
    // kNttKsCombine: component 1's base, limb l of ciphertext ct at
    // d1 + ct d1_ct_stride + l d1_limb (one load path for both components,
    // no branch on the base in the store loop)
    const u64 *d1;
    u64 d1_ct_stride, d1_limb;
};

struct PersistRunner;  // persist.h

// ------------------------------------------------------------ workspace pool

// Caching device allocator.  A released block is handed out again only for
// work on the same stream (stream order makes the reuse safe); the stream is
// the calling thread's current one, set at each C-ABI entry.
extern thread_local hipStream_t tl_stream;

struct Pool {
    std::mutex mu;
    struct Cached {
        void *p;
        uint64_t seq;  // release order, for least-recently-released eviction
    };
    std::multimap<std::pair<hipStream_t, size_t>, Cached> free_;
    uint64_t seq = 0;
    std::map<void *, std::pair<size_t, hipStream_t>> live_;
    size_t held = 0;
    size_t cached = 0;               // bytes of free_ blocks
    size_t limit = 0;                // bytes held (live + cached) beyond which cached blocks are evicted (0: none)
    bool recording = false;          // collect every block handed out (graph capture)
    int64_t fail_after = 0;          // test hook: the n-th next new device allocation fails (0: off)
    std::vector<void *> recorded;
    static size_t size_class(size_t bytes);
    void *alloc(size_t bytes);
    // Removes the recorded blocks (all released by now) from the pool and
    // returns them: a recorded graph keeps using them.
    std::vector<void *> detach_recorded();
    void release(void *p);
    void trim();
    void free_cached();          // caller holds mu
    void evict_to(size_t bytes);  // caller holds mu: oldest releases first, until held <= bytes
    ~Pool();
};

// --------------------------------------------------------------- profiling
// Optional HIP-event bracketing of kernel launches on their own stream.
enum ProfKind {
    kProfNttFwd = 0,
    kProfNttInv = 1,
    kProfNttFwdCombine = 2,
    kProfNttFwdPart = 3,
    kProfNttInvPart = 4,
    kProfTensor = 5,
    kProfModUp = 6,
    kProfKsInner = 7,
    kProfRelinMs = 8,
    kProfLincomb = 9,
    kProfMul = 10,
    kProfKinds = 11
};
struct ProfRec {
    int kind;
    hipEvent_t a, b;
    double bytes;  // algorithmic HBM bytes of the bracketed launches
};
struct Profiler {
    std::mutex mu;
    bool on = false;
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> spare;
    hipEvent_t take();
    void begin(int kind, double bytes, hipStream_t st, ProfRec &r);
    void end(ProfRec &r, hipStream_t st);
    void clear();
    ~Profiler();
};

// ----------------------------------------------------------------- context

// Recorded comparison circuits: one hipGraph per (call, shape, buffers) key,
// with the workspace blocks it was recorded on (owned until destruction).
struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<void *> blocks;
};
struct GraphCache {
    std::map<std::string, GraphEntry> entries;
    ~GraphCache();
};

// ------------------------------------------------------------- noise model
// Host-side estimate of a ciphertext's noise: log2 of a bound on the infinity
// norm of [c0 + c1 s (+ c2 s^2)]_Q (the plaintext included), which must stay
// below Q_l / 2 for the ciphertext to decrypt.  Each operation maps the
// estimates of its inputs to its output's (heuristic: coefficients of the
// products of independent noise polynomials grow with sqrt(N), maxima over
// N coefficients with the Gaussian tail factor sqrt(2 ln 2N)); the constants
// assume the key and encryption randomness the workloads draw (ternary s and
// u, errors of deviation 3.2).  The oracle's exact noise measurement
// calibrates it (the estimate must never be below the measured noise).
struct NoiseModel {
    int N = 0, nQ = 0, nP = 0, dnum = 0, alpha = 0;
    double p = 0, z = 0;
    std::vector<double> lq;   // log2 q_i, i < nQ
    std::vector<double> lQ;   // log2 (q_0 ... q_l)
    double lP = 0;            // log2 P
    NoiseModel() = default;
    NoiseModel(const bc_params &prm, const std::vector<u64> &mod);
    double fresh() const;
    double budget(int level) const { return lQ[level] - 1.0; }  // log2 (Q_l / 2)
    double add(double a, double b) const;
    double scalar(double a, double absc) const;
    double add_const(double a) const;
    // tensor product (three components)
    double tensor(double a, double b) const;
    // key switch (relinearisation or rotation) of a ciphertext with noise t at `level`
    double key_switch(int level, double t) const;
    // relinearised product (plus an addend c, or -inf) at `level`, before the
    // modulus switch
    double product(int level, double a, double b, double c) const;
    // the modulus switch that drops q_level
    double mod_switch(int level, double a) const;
    // automorphism plus key switch at `level`
    double rotate(int level, double a) const;
    // the noise of an input batch (0 = unknown: taken as a fresh encryption's)
    double input(float bits) const { return bits > 0 ? (double)bits : fresh(); }
    // BC_ERR_LEVEL unless `bits` fits the budget of `level`
    void require(int level, double bits, const char *what) const;
};

std::vector<u64> param_moduli(const bc_params &prm);

}  // namespace bc

struct bc_ctx {
    bc_params prm;
    int N, logN, nQ, nP, nmod, dnum, alpha, M;
    bc::u64 p;
    std::vector<bc::u64> mod;  // host copy of the moduli
    bc::NoiseModel noise;
    // device tables
    bc::u64 *tw = nullptr;            // [nmod][4][N]: W, W', Winv, Winv'
    double *twf = nullptr;            // [nmod][4][N]: W, W/q, Winv, Winv/q (all primes < 2^50)
    bc::PrimeInfo *pinfo = nullptr;   // [nmod]
    bc::ModUpPlan *modup = nullptr;   // [nQ][dnum]  (level, digit)
    bc::ModDownPlan *moddown = nullptr;
    bc::ModSwitchPlan *modsw = nullptr;  // [nQ]
    // the same plans with FPair constants (only when every prime < 2^50)
    bc::ModUpPlan *modup_f = nullptr;
    bc::ModDownPlan *moddown_f = nullptr;
    bc::ModSwitchPlan *modsw_f = nullptr;
    bc::GarnerTable *garner = nullptr;
    bc::u64 *zeros = nullptr;  // [N] zero words (the key switch's missing base)
    std::vector<bc::PrimeInfo> h_pinfo;
    std::vector<bc::ModUpPlan> h_modup;  // host copies (launch sizing)
    bc::Pool pool;
    int exec_mode = BC_EXEC_BATCHED;
    size_t ntt_chunk_bytes = 0;  // 0: one launch pair per transform call
    int ntt_single_pass = 1;     // one-launch transform for N = 2^12 .. 2^15
    int ntt_parts = 1;           // N = 2^14, 2^15: producers fold the first stages, parts finish
    int fp64 = 1;                // fp64 transforms and base conversions where twf exists
    std::unique_ptr<bc::GraphCache> graphs;
    std::mutex graph_mu;
    hipStream_t capture_stream = nullptr;      // graph recording (created on first use)
    // a comparison's groups split over `split` library streams forked from
    // and joined back into the caller's stream (created on first use, at the
    // default priority)
    int split = 1;
    std::mutex split_mu;
    std::vector<hipStream_t> split_streams;
    std::vector<hipEvent_t> split_done;
    hipEvent_t split_fork = nullptr;
    std::unique_ptr<bc::Profiler> prof{new bc::Profiler()};
    std::mutex table_mu;                       // guards lt_c and ps_coef
    std::vector<int64_t> lt_c;                 // LT polynomial coefficients
    std::map<int, bc::u64 *> ps_coef;          // block coefficients: per level (pairs), -1 (small ints)
    // bivariate circuit: the weights of g_k(S) and of the final sum, as doubles
    // (one device allocation; built on first use)
    double *biv_tab = nullptr;
    int biv_K = 0, biv_M = 0;
    bool biv_mfma = false;  // the table has the matrix-core copy
    int mfma = 1;           // BC_TUNE_MFMA: use the matrix-core kernels where they apply
    int mfma_modup = 0;     // BC_TUNE_MFMA_MODUP: modulus raising on the matrix cores
    bc::ModUpMfma modup_mfma[3];  // its weight tables, per number of folded stages
    int raw_handoff = 1;    // BC_TUNE_RAW_HANDOFF: key-switching intermediates as reduced fp64 patterns
    // owners: the caller's handle, every live key set and every group that
    // lists the context; the last release deletes it (a key set destroyed
    // after its context's handle still finds the context)
    std::atomic<int> refs{1};
    // comparisons as one persistent launch (BC_TUNE_PERSISTENT), the split
    // slices as lanes; the runner is created on first use
    int persistent = 0;
    std::unique_ptr<bc::PersistRunner> runner;
    int device = 0;                 // current device at creation (every call runs there)
    void *scratch = nullptr;        // that device's allocation-free workspace (device address)
    std::string scratch_err;        // why the lookup failed, if it did
    ~bc_ctx();
};

namespace bc {
// fp64 arithmetic for the transforms and the base conversions: every prime
// below 2^50 (the fp64 tables exist) and not switched off
inline bool use_fp64(const bc_ctx *c) { return c->fp64 && c->twf != nullptr; }
// the polynomial's linear combinations with its small centred coefficients
// as fp64 integers (|c| < p/2 < 2^19 keeps every partial sum exact)
inline bool lincomb_small(const bc_ctx *c) { return use_fp64(c) && c->p < ((u64)1 << 20); }
}  // namespace bc

namespace bc {
// Brackets one launch (or one operation's launches) with the context's
// profiler when it is on.
// Recording of launches for the persistent executor (persist.h): while set,
// launchers record instead of launching and nothing is profiled.
struct Recorder;
extern thread_local Recorder *tl_rec;

struct ProfScope {
    const bc_ctx *c;
    hipStream_t st;
    bool on;
    ProfRec r{};
    ProfScope(const bc_ctx *ctx, int kind, double bytes, hipStream_t s)
        : c(ctx), st(s), on(ctx->prof->on && !tl_rec) {
        if (on) c->prof->begin(kind, bytes, st, r);
    }
    ~ProfScope() {
        if (!on) return;
        try {
            c->prof->end(r, st);
        } catch (...) {
        }
    }
};
}  // namespace bc

struct bc_keys {
    bc_ctx *ctx;
    // process-wide unique id: recorded graphs are cached under it (a host
    // address could be reused by a later key set after this one is freed)
    uint64_t uid = 0;
    int ngal;
    std::vector<int> steps;      // rotation step of each Galois key
    std::vector<bc::u64> gal;    // Galois element
    bc::u64 *s_ntt = nullptr;    // [nmod][N]
    bc::u64 *pk = nullptr;       // [2][nQ][N]
    bc::u64 *rlk = nullptr;      // [dnum][2][nmod][N]
    std::vector<bc::u64 *> gk;   // each [dnum][2][nmod][N]
    std::vector<bc::u32 *> perm; // NTT-domain index map of each Galois key
    ~bc_keys();
};

namespace bc {

// ----------------------------------------------------------- host helpers
u64 h_mulmod(u64 a, u64 b, u64 q);
u64 h_powmod(u64 b, u64 e, u64 q);
u64 h_invmod(u64 a, u64 q);
inline u64 h_shoup(u64 w, u64 q) { return (u64)(((u128)w << 64) / q); }
// (w, w/q) as doubles in the two words of a pair (fp64 arithmetic, q < 2^50;
// the quotient is correctly rounded)
inline void h_fpair(u64 dst[2], u64 w, u64 q) {
    const double wd = (double)(w % q), r = wd / (double)q;
    std::memcpy(&dst[0], &wd, sizeof(double));
    std::memcpy(&dst[1], &r, sizeof(double));
}
int bit_reverse(int x, int bits);

// ----------------------------------------------------------------- kernels
void ntt_forward(const bc_ctx *c, const LimbSet &ls, hipStream_t st);
void ntt_inverse(const bc_ctx *c, const LimbSet &ls, hipStream_t st);
// Forward transform of E with the NttCombine step as its epilogue (E itself
// is not written back).  Returns false, launching nothing, when the context's
// transform schedule has no such kernel; the caller then transforms E and
// combines separately (same result).
bool ntt_forward_combine(const bc_ctx *c, const LimbSet &ls, const NttCombine &cb, hipStream_t st);
// Part-limb forward transforms.  When PL = ntt_parts_log(c) > 0 (N = 2^14:
// 1, N = 2^15: 2), the kernels that produce words for the key-switching
// transforms (modulus raising, the relinearise+switch and switch corrections)
// apply the transform's first PL butterfly stages themselves (fold_int /
// fold_fp), and these finish it in 2^PL independent parts of 2^13 words: one
// block of 256 threads each, four blocks per CU.
int ntt_parts_log(const bc_ctx *c);
void ntt_forward_parts(const bc_ctx *c, const LimbSet &ls, hipStream_t st);
void ntt_forward_parts_combine(const bc_ctx *c, const LimbSet &ls, const NttCombine &cb, hipStream_t st);
// Inverse transform of every part of each limb except its last PL stages,
// which the kernel that consumes the words applies (unfold_int / unfold_fp):
// modulus raising, and the relinearise+switch and switch corrections.
void ntt_inverse_parts(const bc_ctx *c, const LimbSet &ls, hipStream_t st);

}  // namespace bc
