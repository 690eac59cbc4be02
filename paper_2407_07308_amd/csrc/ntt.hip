// ntt.hip -- batched negacyclic NTT / inverse NTT for gfx950.
//
// The residue polynomials of a ciphertext are multiplied in the evaluation
// domain (paper, Background, "Efficient Polynomial and NTT": radix-2
// Cooley-Tukey forward and Gentleman-Sande inverse transforms for power-of-two
// N).  Forward: natural-order coefficients in, bit-reversed evaluations out,
// position r holding a(psi^(2 brv(r) + 1)); the stage with butterfly span h
// (m = N / 2h) multiplies group i by W[m + i] = psi^brv(m + i).  Inverse:
// Gentleman-Sande with Winv[k] = W[k]^-1 in the reverse stage order, scaled
// by N^-1.
//
// A limb of N = N1 * N2 words is an N1 x N2 row-major matrix.  The forward
// stages with span >= N2 only mix words of one column (pass A), the others
// only words of one row (pass B); the inverse runs B then A.  Each pass reads
// and writes every word of the limb once.  Inside a pass the line (column or
// row) is transformed in two register chunks of up to four stages: a thread
// holds up to 16 words, applies its chunk's butterflies in registers, and the
// two chunks exchange words through LDS once.  The butterflies' arithmetic
// is a policy: integer (Harvey's lazy butterflies with Shoup products) for
// any prime, or fp64 for primes below 2^50 (see FpA).

#include <type_traits>

#include "ntt_dev.h"
#include "persist.h"

namespace bc {

namespace {

template <int LOGN, bool INV, class A>
__global__ void __launch_bounds__(1 << (LOGN - 5)) ntt_full(LimbSet ls, const void *__restrict__ tw,
                                                            const PrimeInfo *__restrict__ pinfo) {
    __shared__ u64 s[ntt_lds_words(LOGN, 0)];
    ntt_full_body<LOGN, INV, A, 0>(ls, tw, pinfo, nullptr, blockIdx.x, s);
}

// Parts of 2^(LOGN+PL)-word limbs (2^PL blocks per limb, block 2^PL job +
// part), several blocks per CU: four waves per SIMD (128 registers a lane)
// forward; three inverse, whose chunks need more registers (timed faster
// than four with spills).
template <int LOGN, class A, int PL = 1, bool INV = false, bool RIN = false, bool ROUT = false>
__global__ void __launch_bounds__(1 << (LOGN - 5), INV ? 3 : 4) ntt_part(LimbSet ls, const void *__restrict__ tw,
                                                                         const PrimeInfo *__restrict__ pinfo) {
    __shared__ u64 s[ntt_lds_words(LOGN, PL)];
    ntt_full_body<LOGN, INV, A, 0, PL, false, RIN, ROUT>(ls, tw, pinfo, nullptr, blockIdx.x, s);
}
template <int LOGN, class A, int EPI, int PL = 1, bool RIN = false>
__global__ void __launch_bounds__(1 << (LOGN - 5), 4)
    ntt_part_combine(LimbSet ls, const void *__restrict__ tw, const PrimeInfo *__restrict__ pinfo, NttCombine cb) {
    __shared__ u64 s[ntt_lds_words(LOGN, PL)];
    ntt_full_body<LOGN, false, A, EPI, PL, false, RIN>(ls, tw, pinfo, &cb, blockIdx.x, s);
}

// forward transform of E limbs with an NttCombine step as the store (out
// gets the combination; E is not written back)
template <int LOGN, class A, int EPI>
__global__ void __launch_bounds__(1 << (LOGN - 5)) ntt_full_combine(LimbSet ls, const void *__restrict__ tw,
                                                                    const PrimeInfo *__restrict__ pinfo,
                                                                    NttCombine cb) {
    __shared__ u64 s[ntt_lds_words(LOGN, 0)];
    ntt_full_body<LOGN, false, A, EPI>(ls, tw, pinfo, &cb, blockIdx.x, s);
}

// Arithmetic of a context's transforms: fp64 when every prime allows it and
// it is enabled, else the integer butterflies.
inline bool use_fp(const bc_ctx *c) { return use_fp64(c); }
inline const void *tw_of(const bc_ctx *c) { return use_fp(c) ? (const void *)c->twf : (const void *)c->tw; }

// Records a transform stage for the persistent executor: 2^13-word blocks
// (whole limbs at N = 2^13, halves at 2^14, quarters at 2^15), fp64.
void record_ntt(const bc_ctx *c, const LimbSet &ls, int kind0, int pl, const NttCombine *cb) {
    BC_REQUIRE(!ls.raw_in && !ls.raw_out, BC_ERR_ARG, "the persistent executor passes canonical words");
    BC_REQUIRE(use_fp(c), BC_ERR_ARG, "the persistent executor needs fp64 arithmetic");
    BC_REQUIRE(c->logN - pl == 13, BC_ERR_ARG,
               "the persistent executor runs 2^13-word transform blocks (N = 2^13, or part-limb at 2^14 and 2^15)");
    BC_REQUIRE(!cb || cb->mode == kNttRelinMs, BC_ERR_ARG, "the persistent executor combines relinearisation only");
    PaNtt a{};
    a.ls = ls;
    a.tw = tw_of(c);
    a.pinfo = c->pinfo;
    if (cb) a.cb = *cb;
    // kinds come in (forward, inverse, combine) triples per pl
    tl_rec->add(kind0 + 3 * pl, dim3((unsigned)(ls.npoly * ls.nlimb) << pl, 1, 1), a, 1);
}

template <bool INV, class A>
bool launch_full_a(int logN, const LimbSet &ls, const bc_ctx *c, hipStream_t st) {
    const unsigned njobs = (unsigned)(ls.npoly * ls.nlimb);
#define BC_FULL(L)                                                                                \
    case L:                                                                                       \
        ntt_full<L, INV, A><<<njobs, 1 << (L - 5), 0, st>>>(ls, tw_of(c), c->pinfo);              \
        return true;
    switch (logN) {
        BC_FULL(12) BC_FULL(13) BC_FULL(14) BC_FULL(15)
        default: return false;
    }
#undef BC_FULL
}

template <bool INV>
bool launch_full(int logN, const LimbSet &ls, const bc_ctx *c, hipStream_t st) {
    return use_fp(c) ? launch_full_a<INV, FpA>(logN, ls, c, st) : launch_full_a<INV, IntA>(logN, ls, c, st);
}

template <bool INV, class A>
void launch_cols_a(int logN1, int logN, const LimbSet &ls, const bc_ctx *c, hipStream_t st) {
    int N2 = 1 << (logN - logN1), C = cols_per_block(logN1);
    int njobs = ls.npoly * ls.nlimb;
    dim3 grid((unsigned)(njobs * (N2 / C)));
#define BC_COLS(L)                                                                                \
    case L:                                                                                       \
        ntt_cols<L, INV, A><<<grid, kThreads, 0, st>>>(ls, tw_of(c), c->pinfo, logN);             \
        break;
    switch (logN1) {
        BC_COLS(5) BC_COLS(6) BC_COLS(7) BC_COLS(8)
        default: throw Error(BC_ERR_PARAM, "ntt: unsupported column length");
    }
#undef BC_COLS
}

template <bool INV>
void launch_cols(int logN1, int logN, const LimbSet &ls, const bc_ctx *c, hipStream_t st) {
    if (use_fp(c)) launch_cols_a<INV, FpA>(logN1, logN, ls, c, st);
    else launch_cols_a<INV, IntA>(logN1, logN, ls, c, st);
}

template <bool INV, class A>
void launch_rows_a(int logN2, int logN, const LimbSet &ls, const bc_ctx *c, hipStream_t st) {
    int N1 = 1 << (logN - logN2), R = std::min(kLineWords >> logN2, N1);
    int njobs = ls.npoly * ls.nlimb;
    dim3 grid((unsigned)(njobs * (N1 / R)));
#define BC_ROWS(L)                                                                                \
    case L:                                                                                       \
        ntt_rows<L, INV, A><<<grid, kThreads, 0, st>>>(ls, tw_of(c), c->pinfo, logN);             \
        break;
    switch (logN2) {
        BC_ROWS(5) BC_ROWS(6) BC_ROWS(7) BC_ROWS(8)
        default: throw Error(BC_ERR_PARAM, "ntt: unsupported row length");
    }
#undef BC_ROWS
}

template <bool INV>
void launch_rows(int logN2, int logN, const LimbSet &ls, const bc_ctx *c, hipStream_t st) {
    if (use_fp(c)) launch_rows_a<INV, FpA>(logN2, logN, ls, c, st);
    else launch_rows_a<INV, IntA>(logN2, logN, ls, c, st);
}

}  // namespace

// Algorithmic bytes of a transform: every limb read once and written once.
static double ntt_bytes(const bc_ctx *c, const LimbSet &ls) { return 16.0 * c->N * ls.npoly * ls.nlimb; }

// Polynomials per launch pair: with a chunk size set, the two passes run on
// slices of at most that many bytes, so the intermediate written by the first
// pass can still sit in the 256 MB last-level cache when the second reads it.
static int polys_per_chunk(const bc_ctx *c, const LimbSet &ls) {
    const size_t per_poly = (size_t)ls.nlimb * 8 * c->N;
    if (c->ntt_chunk_bytes == 0 || ls.poly_stride == 0) return ls.npoly;
    return (int)std::max<size_t>(1, c->ntt_chunk_bytes / per_poly);
}

// Polys [p0, p0 + step) of a limb set.
static LimbSet chunk_of(const LimbSet &ls, int p0, int step) {
    LimbSet sub = ls;
    sub.base = ls.base + (size_t)p0 * ls.poly_stride;
    if (ls.ibase) sub.ibase = ls.ibase + (size_t)p0 * ls.ipoly_stride;
    sub.npoly = std::min(step, ls.npoly - p0);
    return sub;
}

// N1 = 2^floor(logN/2) rows, N2 = 2^ceil(logN/2) columns.
void ntt_forward(const bc_ctx *c, const LimbSet &ls, hipStream_t st) {
    if (ls.npoly == 0 || ls.nlimb == 0) return;
    if (tl_rec) return record_ntt(c, ls, kPkNttFwd0, 0, nullptr);
    int logN1 = c->logN / 2, logN2 = c->logN - logN1;
    ProfRec r{};
    const bool prof = c->prof->on && !tl_rec;
    if (prof) c->prof->begin(kProfNttFwd, ntt_bytes(c, ls), st, r);
    if (c->ntt_single_pass && launch_full<false>(c->logN, ls, c, st)) {
        if (prof) c->prof->end(r, st);
        BC_HIP(hipGetLastError());
        return;
    }
    const int step = polys_per_chunk(c, ls);
    for (int p0 = 0; p0 < ls.npoly; p0 += step) {
        LimbSet sub = chunk_of(ls, p0, step);
        launch_cols<false>(logN1, c->logN, sub, c, st);
        sub.ibase = nullptr;  // the second pass works in place on the output
        launch_rows<false>(logN2, c->logN, sub, c, st);
    }
    if (prof) c->prof->end(r, st);
    BC_HIP(hipGetLastError());
}

void ntt_inverse(const bc_ctx *c, const LimbSet &ls, hipStream_t st) {
    if (ls.npoly == 0 || ls.nlimb == 0) return;
    if (tl_rec) return record_ntt(c, ls, kPkNttInv0, 0, nullptr);
    int logN1 = c->logN / 2, logN2 = c->logN - logN1;
    ProfRec r{};
    const bool prof = c->prof->on && !tl_rec;
    if (prof) c->prof->begin(kProfNttInv, ntt_bytes(c, ls), st, r);
    if (c->ntt_single_pass && launch_full<true>(c->logN, ls, c, st)) {
        if (prof) c->prof->end(r, st);
        BC_HIP(hipGetLastError());
        return;
    }
    const int step = polys_per_chunk(c, ls);
    for (int p0 = 0; p0 < ls.npoly; p0 += step) {
        LimbSet sub = chunk_of(ls, p0, step);
        launch_rows<true>(logN2, c->logN, sub, c, st);
        sub.ibase = nullptr;  // the second pass works in place on the output
        launch_cols<true>(logN1, c->logN, sub, c, st);
    }
    if (prof) c->prof->end(r, st);
    BC_HIP(hipGetLastError());
}

template <class A, int EPI>
static bool launch_full_combine(int logN, const LimbSet &ls, const NttCombine &cb, const bc_ctx *c, hipStream_t st) {
    const unsigned njobs = (unsigned)(ls.npoly * ls.nlimb);
#define BC_FULL_CB(L)                                                                             \
    case L:                                                                                       \
        ntt_full_combine<L, A, EPI><<<njobs, 1 << (L - 5), 0, st>>>(ls, tw_of(c), c->pinfo, cb);  \
        return true;
    switch (logN) {
        BC_FULL_CB(12) BC_FULL_CB(13) BC_FULL_CB(14) BC_FULL_CB(15)
        default: return false;
    }
#undef BC_FULL_CB
}

template <class A>
static bool launch_full_combine_a(int logN, const LimbSet &ls, const NttCombine &cb, const bc_ctx *c,
                                  hipStream_t st) {
    return cb.mode == kNttRelinMs    ? launch_full_combine<A, kNttRelinMs>(logN, ls, cb, c, st)
           : cb.mode == kNttKsCombine ? launch_full_combine<A, kNttKsCombine>(logN, ls, cb, c, st)
                                      : launch_full_combine<A, kNttSwitch>(logN, ls, cb, c, st);
}

// ----------------------------------------------------------- part limbs
// Forward transforms whose first PL stages the producer of the words applied:
// 2^PL blocks of 2^13 words per limb.
int ntt_parts_log(const bc_ctx *c) {
    if (!c->ntt_single_pass || !c->ntt_parts || c->alpha > kFoldDigit || c->nP > kFoldDigit) return 0;
    return c->logN == 15 ? 2 : c->logN == 14 ? 1 : 0;
}

// the part-limb kernel for the limb set's word forms (reduced fp64 patterns
// only with fp64 arithmetic)
template <class A, bool INV>
static void launch_parts_k(int pl, const LimbSet &ls, const bc_ctx *c, hipStream_t st) {
    const unsigned nblk = (unsigned)(ls.npoly * ls.nlimb) << pl;
    auto go = [&](auto rin, auto rout) {
        constexpr bool RI = decltype(rin)::value, RO = decltype(rout)::value;
        if (pl == 2) ntt_part<13, A, 2, INV, RI, RO><<<nblk, 256, 0, st>>>(ls, tw_of(c), c->pinfo);
        else ntt_part<13, A, 1, INV, RI, RO><<<nblk, 256, 0, st>>>(ls, tw_of(c), c->pinfo);
    };
    if constexpr (A::kDerive) {
        if (ls.raw_in && ls.raw_out) go(std::true_type{}, std::true_type{});
        else if (ls.raw_in) go(std::true_type{}, std::false_type{});
        else if (ls.raw_out) go(std::false_type{}, std::true_type{});
        else go(std::false_type{}, std::false_type{});
    } else {
        BC_REQUIRE(!ls.raw_in && !ls.raw_out, BC_ERR_ARG, "reduced fp64 words need the fp64 arithmetic");
        go(std::false_type{}, std::false_type{});
    }
}
template <class A>
static void launch_parts(int pl, const LimbSet &ls, const bc_ctx *c, hipStream_t st) {
    launch_parts_k<A, false>(pl, ls, c, st);
}

void ntt_forward_parts(const bc_ctx *c, const LimbSet &ls, hipStream_t st) {
    const int pl = ntt_parts_log(c);
    if (!pl) throw Error(BC_ERR_ARG, "ntt: part-limb transforms are off for this context");
    if (ls.npoly == 0 || ls.nlimb == 0) return;
    if (tl_rec) return record_ntt(c, ls, kPkNttFwd0, pl, nullptr);
    ProfRec r{};
    const bool prof = c->prof->on && !tl_rec;
    if (prof) c->prof->begin(kProfNttFwdPart, ntt_bytes(c, ls), st, r);
    if (use_fp(c)) launch_parts<FpA>(pl, ls, c, st);
    else launch_parts<IntA>(pl, ls, c, st);
    if (prof) c->prof->end(r, st);
    BC_HIP(hipGetLastError());
}

template <class A>
static void launch_parts_inv(int pl, const LimbSet &ls, const bc_ctx *c, hipStream_t st) {
    launch_parts_k<A, true>(pl, ls, c, st);
}

void ntt_inverse_parts(const bc_ctx *c, const LimbSet &ls, hipStream_t st) {
    const int pl = ntt_parts_log(c);
    if (!pl) throw Error(BC_ERR_ARG, "ntt: part-limb transforms are off for this context");
    if (ls.npoly == 0 || ls.nlimb == 0) return;
    if (tl_rec) return record_ntt(c, ls, kPkNttInv0, pl, nullptr);
    ProfRec r{};
    const bool prof = c->prof->on && !tl_rec;
    if (prof) c->prof->begin(kProfNttInvPart, ntt_bytes(c, ls), st, r);
    if (use_fp(c)) launch_parts_inv<FpA>(pl, ls, c, st);
    else launch_parts_inv<IntA>(pl, ls, c, st);
    if (prof) c->prof->end(r, st);
    BC_HIP(hipGetLastError());
}

template <class A, int EPI>
static void launch_parts_combine(int pl, const LimbSet &ls, const NttCombine &cb, const bc_ctx *c, hipStream_t st) {
    const unsigned nblk = (unsigned)(ls.npoly * ls.nlimb) << pl;
    BC_REQUIRE(!ls.raw_out, BC_ERR_ARG, "a combined transform stores canonical words");
    auto go = [&](auto rin) {
        constexpr bool RI = decltype(rin)::value;
        if (pl == 2) ntt_part_combine<13, A, EPI, 2, RI><<<nblk, 256, 0, st>>>(ls, tw_of(c), c->pinfo, cb);
        else ntt_part_combine<13, A, EPI, 1, RI><<<nblk, 256, 0, st>>>(ls, tw_of(c), c->pinfo, cb);
    };
    if constexpr (A::kDerive) {
        if (ls.raw_in) go(std::true_type{});
        else go(std::false_type{});
    } else {
        BC_REQUIRE(!ls.raw_in, BC_ERR_ARG, "reduced fp64 words need the fp64 arithmetic");
        go(std::false_type{});
    }
}

template <class A>
static void launch_parts_combine_a(int pl, const LimbSet &ls, const NttCombine &cb, const bc_ctx *c,
                                   hipStream_t st) {
    if (cb.mode == kNttRelinMs) launch_parts_combine<A, kNttRelinMs>(pl, ls, cb, c, st);
    else if (cb.mode == kNttKsCombine) launch_parts_combine<A, kNttKsCombine>(pl, ls, cb, c, st);
    else launch_parts_combine<A, kNttSwitch>(pl, ls, cb, c, st);
}

void ntt_forward_parts_combine(const bc_ctx *c, const LimbSet &ls, const NttCombine &cb, hipStream_t st) {
    const int pl = ntt_parts_log(c);
    if (!pl) throw Error(BC_ERR_ARG, "ntt: part-limb transforms are off for this context");
    if (cb.mode != kNttRelinMs && cb.mode != kNttSwitch && cb.mode != kNttKsCombine)
        throw Error(BC_ERR_ARG, "ntt: unknown combine step");
    if (ls.npoly == 0 || ls.nlimb == 0) return;
    if (tl_rec) return record_ntt(c, ls, kPkNttComb0, pl, &cb);
    ProfRec r{};
    const bool prof = c->prof->on && !tl_rec;
    const double per_limb = (cb.mode == kNttRelinMs ? 32.0 : cb.mode == kNttKsCombine ? 28.0 : 24.0) * c->N;
    if (prof) c->prof->begin(kProfNttFwdCombine, per_limb * ls.npoly * ls.nlimb, st, r);
    if (use_fp(c)) launch_parts_combine_a<FpA>(pl, ls, cb, c, st);
    else launch_parts_combine_a<IntA>(pl, ls, cb, c, st);
    if (prof) c->prof->end(r, st);
    BC_HIP(hipGetLastError());
}

bool ntt_forward_combine(const bc_ctx *c, const LimbSet &ls, const NttCombine &cb, hipStream_t st) {
    if (!c->ntt_single_pass || c->logN < 12 || c->logN > 15) return false;
    if (cb.mode != kNttRelinMs && cb.mode != kNttSwitch && cb.mode != kNttKsCombine)
        throw Error(BC_ERR_ARG, "ntt: unknown combine step");
    if (ls.npoly == 0 || ls.nlimb == 0) return true;
    if (tl_rec) {
        record_ntt(c, ls, kPkNttComb0, 0, &cb);
        return true;
    }
    ProfRec r{};
    const bool prof = c->prof->on && !tl_rec;
    // E read and out written, d (and acc) read
    const double per_limb = (cb.mode == kNttRelinMs ? 32.0 : cb.mode == kNttKsCombine ? 28.0 : 24.0) * c->N;
    if (prof) c->prof->begin(kProfNttFwdCombine, per_limb * ls.npoly * ls.nlimb, st, r);
    const bool ok = use_fp(c) ? launch_full_combine_a<FpA>(c->logN, ls, cb, c, st)
                              : launch_full_combine_a<IntA>(c->logN, ls, cb, c, st);
    if (prof) c->prof->end(r, st);
    BC_HIP(hipGetLastError());
    return ok;
}

}  // namespace bc
