// kernels.hip -- element-wise, base-conversion and key-switching kernels.
//
// Every ciphertext limb is a contiguous run of N uint64 residues; a batch is
// [count][ncomp][nlimb][N].  Kernels use a 3-D grid: x covers the N
// coefficients of a limb (256 per workgroup, fully coalesced), y the limb, z
// the ciphertext of the batch, so no kernel divides by a runtime size.  These
// are the element-wise operations the paper offloads as whole residue
// matrices (paper, "GPU-related Optimizations": one launch over the
// (L+1) x N matrix instead of one per row), plus the base conversions of
// hybrid key switching and modulus switching.

#include <type_traits>

#include "kernels.h"
#include "kernels_dev.h"
#include "persist.h"

namespace bc {

namespace {


// ------------------------------------------------------------ ring ops

template <bool ADD>
__global__ void k_tensor(const u64 *__restrict__ a, const u64 *__restrict__ b, const u64 *__restrict__ c,
                         u64 *__restrict__ out, int bcount, int nl, int na, int nb, int nc,
                         const PrimeInfo *__restrict__ pinfo, int N) {
    b_tensor<ADD>(hw_blk(), a, b, c, out, bcount, nl, na, nb, nc, pinfo, N);
}

__global__ void k_addsub(const u64 *__restrict__ a, const u64 *__restrict__ b, u64 *__restrict__ out, int bcount,
                         int nl, int na, int nb, int ncomp, int sub, const PrimeInfo *__restrict__ pinfo, int N) {
    b_addsub(hw_blk(), a, b, out, bcount, nl, na, nb, ncomp, sub, pinfo, N);
}


__global__ void k_mul_scalar(const u64 *__restrict__ a, u64 *__restrict__ out, int nl, int ncomp, ScalarArg s,
                             const PrimeInfo *__restrict__ pinfo, int N) {
    b_mul_scalar(hw_blk(), a, out, nl, ncomp, s, pinfo, N);
}

__global__ void k_add_const(const u64 *__restrict__ a, u64 *__restrict__ out, int nl, int ncomp, ScalarArg s,
                            const PrimeInfo *__restrict__ pinfo, int N) {
    b_add_const(hw_blk(), a, out, nl, ncomp, s, pinfo, N);
}

__global__ void k_mul_monomial(const u64 *__restrict__ a, u64 *__restrict__ out, int nl, int ncomp, int e,
                               const u64 *__restrict__ tw, const PrimeInfo *__restrict__ pinfo, int N, int logN) {
    b_mul_monomial(hw_blk(), a, out, nl, ncomp, e, tw, pinfo, N, logN);
}

__global__ void k_permute(const u64 *__restrict__ in, u64 *__restrict__ out, const u32 *__restrict__ perm, int nl,
                          int ncomp, int N, const PrimeInfo *__restrict__ pinfo, bool add0) {
    b_permute(hw_blk(), in, out, perm, nl, ncomp, N, pinfo, add0);
}

// ------------------------------------------------------- key switching

template <bool FP, int PL = 0, int MD = kMaxDigit, bool RAW = false>
__global__ void k_modup(const u64 *__restrict__ xc, u64 *__restrict__ mu, const ModUpPlan *__restrict__ plans,
                        const PrimeInfo *__restrict__ pinfo, int nl, int next, int dnum, int N) {
    b_modup<FP, PL, MD, RAW>(hw_blk(), xc, mu, plans, pinfo, nl, next, dnum, N);
}

template <bool FP, bool RAW = false>
__global__ void k_ks_inner(const u64 *__restrict__ mu, const u64 *__restrict__ x, size_t x_ct_stride,
                           const u64 *__restrict__ key, u64 *__restrict__ acc, int level, int nQ, int nmod, int next,
                           int nact, int dnum, int alpha, int count, const PrimeInfo *__restrict__ pinfo, int N) {
    b_ks_inner<FP, RAW>(hw_blk(), mu, x, x_ct_stride, key, acc, level, nQ, nmod, next, nact, dnum, alpha, count, pinfo,
                        N);
}

template <bool FP, int PL, bool SC = false>
__global__ void k_moddown(const u64 *__restrict__ acc, u64 *__restrict__ th, const ModDownPlan *__restrict__ pl,
                          const PrimeInfo *__restrict__ pinfo, int level, int nQ, int nP, int next, int N) {
    b_moddown<FP, PL, SC>(hw_blk(), acc, th, pl, pinfo, level, nQ, nP, next, N);
}

__global__ void k_ks_combine(const u64 *__restrict__ base0, const u64 *__restrict__ base1, size_t base_ct_stride,
                             const u64 *__restrict__ acc, const u64 *__restrict__ th, u64 *__restrict__ out,
                             size_t out_ct_stride, const ModDownPlan *__restrict__ pl,
                             const PrimeInfo *__restrict__ pinfo, int nl, int next, int N) {
    b_ks_combine(hw_blk(), base0, base1, base_ct_stride, acc, th, out, out_ct_stride, pl, pinfo, nl, next, N);
}

template <bool FP, int PL = 0, int MD = kMaxDigit, bool RAW = false>
__global__ void k_relin_ms_fbc(const u64 *__restrict__ acc, const u64 *__restrict__ d, size_t d_ct_stride,
                               u64 *__restrict__ E, const ModDownPlan *__restrict__ md,
                               const ModSwitchPlan *__restrict__ ms, const PrimeInfo *__restrict__ pinfo, int level,
                               int nQ, int nP, int next, int N) {
    b_relin_ms_fbc<FP, PL, MD, RAW>(hw_blk(), acc, d, d_ct_stride, E, md, ms, pinfo, level, nQ, nP, next, N);
}

// out[ct][c][i] = (d_i + acc_i P^-1) q_l^-1 - E_i, i < level (NTT domain)
struct PairArg {
    u64 w[kMaxMod][4];  // q_l^-1 and P^-1 q_l^-1 mod q_i (Shoup pairs)
};
__global__ void k_relin_ms_combine(const u64 *__restrict__ d, size_t d_ct_stride, const u64 *__restrict__ acc,
                                   const u64 *__restrict__ E, u64 *__restrict__ out, PairArg pa,
                                   const PrimeInfo *__restrict__ pinfo, int level, int next, int N) {
    const int n = blockIdx.x * kT + threadIdx.x, i = blockIdx.y, ct = blockIdx.z;
    const u64 q = pinfo[i].q;
    const int nl = level + 1;
    for (int c = 0; c < 2; c++) {
        u64 x = shoup(d[(size_t)ct * d_ct_stride + ((size_t)c * nl + i) * N + n], pa.w[i][0], pa.w[i][1], q);
        u64 y = shoup(acc[(((size_t)ct * 2 + c) * next + i) * N + n], pa.w[i][2], pa.w[i][3], q);
        u64 e = E[(((size_t)ct * 2 + c) * level + i) * N + n];
        out[(((size_t)ct * 2 + c) * level + i) * N + n] = sub_mod(add_mod(x, y, q), e, q);
    }
}

// ----------------------------------------------------- modulus switching

template <bool FP, int PL = 0>
__global__ void k_ms_fbc(const u64 *__restrict__ top, u64 *__restrict__ R, const ModSwitchPlan *__restrict__ pl,
                         const PrimeInfo *__restrict__ pinfo, int level, int N) {
    b_ms_fbc<FP, PL>(hw_blk(), top, R, pl, pinfo, level, N);
}

__global__ void k_ms_combine(const u64 *__restrict__ in, const u64 *__restrict__ R, u64 *__restrict__ out,
                             const ModSwitchPlan *__restrict__ pl, const PrimeInfo *__restrict__ pinfo, int level,
                             int N) {
    b_ms_combine(hw_blk(), in, R, out, pl, pinfo, level, N);
}

// -------------------------------------------------------- client side

// words mod q_prime(limb) for a [npoly][nlimb][N] block of raw words
// (Shoup reduction by 1 with floor(2^64 / q), valid for any 64-bit word)
__global__ void k_words_mod(const u64 *__restrict__ w, u64 *__restrict__ out, const int16_t *__restrict__ primes,
                            const PrimeInfo *__restrict__ pinfo, int nlimb, int N) {
    const int n = blockIdx.x * kT + threadIdx.x, k = blockIdx.y, poly = blockIdx.z;
    const u64 q = pinfo[primes[k]].q;
    const u64 wp = (~(u64)0) / q;  // = floor(2^64 / q) for odd q
    size_t off = ((size_t)poly * nlimb + k) * N + n;
    out[off] = shoup(w[off], 1, wp, q);
}

// factor * v (signed small integers, poly `poly` at v + poly * vstride) mod
// q_prime(limb), plus an optional uint32 addend (message coefficients)
__global__ void k_lift_small(const int32_t *__restrict__ v32, const int8_t *__restrict__ v8, size_t vstride,
                             const uint32_t *__restrict__ add, u64 *__restrict__ out, const int16_t *__restrict__ primes,
                             const PrimeInfo *__restrict__ pinfo, int nlimb, int use_p, int N) {
    const int n = blockIdx.x * kT + threadIdx.x, k = blockIdx.y, poly = blockIdx.z;
    const PrimeInfo &pi = pinfo[primes[k]];
    const u64 q = pi.q;
    int64_t x = v32 ? (int64_t)v32[(size_t)poly * vstride + n] : (int64_t)v8[(size_t)poly * vstride + n];
    u64 r = x >= 0 ? (u64)x : q - (u64)(-x);
    if (use_p) r = shoup(r, pi.p_mod, pi.p_modp, q);
    if (add) r = add_mod(r, (u64)add[(size_t)poly * N + n] % q, q);
    out[((size_t)poly * nlimb + k) * N + n] = r;
}

// switching-key pair for one digit: k0 = -A S + E + f S', k1 = A  (NTT domain)
struct FArg {
    u64 f[kMaxMod];  // P mod q_i for the digit's primes, 0 elsewhere
};
__global__ void k_keypair(const u64 *__restrict__ A, const u64 *__restrict__ E, const u64 *__restrict__ S,
                          const u64 *__restrict__ S2, FArg f, u64 *__restrict__ k0, u64 *__restrict__ k1,
                          const PrimeInfo *__restrict__ pinfo, int N) {
    const int n = blockIdx.x * kT + threadIdx.x, i = blockIdx.y;
    const Barrett br = pinfo[i].br;
    size_t off = (size_t)i * N + n;
    u64 a = A[off];
    u64 r = sub_mod(E[off], mul_mod(a, S[off], br), br.q);
    if (S2 && f.f[i]) r = add_mod(r, mul_mod(f.f[i], S2[off], br), br.q);
    k0[off] = r;
    k1[off] = a;
}

// pointwise product of two [nlimb][N] blocks
__global__ void k_pmul(const u64 *__restrict__ a, const u64 *__restrict__ b, u64 *__restrict__ out,
                       const PrimeInfo *__restrict__ pinfo, int N) {
    const int n = blockIdx.x * kT + threadIdx.x, i = blockIdx.y;
    size_t off = (size_t)i * N + n;
    out[off] = mul_mod(a[off], b[off], pinfo[i].br);
}

// c0 = pk0 U + E0, c1 = pk1 U + E1 with U, E0, E1 each [count][nQ][N]
__global__ void k_enc_combine(const u64 *__restrict__ pk, const u64 *__restrict__ U, const u64 *__restrict__ E0,
                              const u64 *__restrict__ E1, u64 *__restrict__ out, int nQ,
                              const PrimeInfo *__restrict__ pinfo, int N) {
    const int n = blockIdx.x * kT + threadIdx.x, i = blockIdx.y, ct = blockIdx.z;
    const Barrett br = pinfo[i].br;
    const size_t L = (size_t)nQ * N, off = (size_t)i * N + n, x = (size_t)ct * L + off;
    u64 u = U[x];
    out[(size_t)ct * 2 * L + off] = add_mod(mul_mod(pk[off], u, br), E0[x], br.q);
    out[(size_t)ct * 2 * L + L + off] = add_mod(mul_mod(pk[L + off], u, br), E1[x], br.q);
}

// D[ct][i] = c0 + c1 s (+ c2 s^2)   (NTT domain)
__global__ void k_dec_inner(const u64 *__restrict__ ct_in, const u64 *__restrict__ s, u64 *__restrict__ d, int nl,
                            int ncomp, const PrimeInfo *__restrict__ pinfo, int N) {
    const int n = blockIdx.x * kT + threadIdx.x, i = blockIdx.y, ct = blockIdx.z;
    const Barrett br = pinfo[i].br;
    const size_t L = (size_t)nl * N, off = (size_t)i * N + n;
    const u64 *C = ct_in + (size_t)ct * ncomp * L;
    u64 sv = s[off], r = C[off], sp = sv;
    for (int k = 1; k < ncomp; k++) {
        r = add_mod(r, mul_mod(C[k * L + off], sp, br), br.q);
        sp = mul_mod(sp, sv, br);
    }
    d[(size_t)ct * L + off] = r;
}

// Garner mixed radix x = v_0 + v_1 q_0 + ...; centred against (Q-1)/2 (whose
// digits are (q_i - 1)/2); result x mod p or (x - Q) mod p.
__global__ void k_crt_decode(const u64 *__restrict__ d, uint32_t *__restrict__ out, const GarnerTable *__restrict__ g,
                             const PrimeInfo *__restrict__ pinfo, int nl, u64 p, int N) {
    const int n = blockIdx.x * kT + threadIdx.x, ct = blockIdx.z;
    u64 v[kMaxMod];
    for (int i = 0; i < nl; i++) {
        const u64 q = pinfo[i].q;
        u64 t = d[((size_t)ct * nl + i) * N + n];
        for (int j = 0; j < i; j++) {
            u64 vj = shoup(v[j], 1, g->one_p[i], q);  // v_j mod q_i
            t = shoup(sub_mod(t, vj, q), g->inv[i][j][0], g->inv[i][j][1], q);
        }
        v[i] = t;
    }
    int cmp = 0;  // sign of x - (Q-1)/2
    for (int i = nl - 1; i >= 0 && cmp == 0; i--) {
        u64 h = (pinfo[i].q - 1) / 2;
        cmp = v[i] > h ? 1 : (v[i] < h ? -1 : 0);
    }
    u64 r = 0;
    for (int i = 0; i < nl; i++) r = (r + (v[i] % p) * g->mprod_p[i]) % p;
    if (cmp > 0) r = (r + p - g->qprod_p[nl - 1]) % p;
    out[(size_t)ct * N + n] = (uint32_t)r;
}

template <bool FP>
__global__ void k_lincomb(BabyArg ba, const u64 *__restrict__ coef, u64 *__restrict__ out, int nbaby, int nblk,
                          int count, int ct0, int nl, const PrimeInfo *__restrict__ pinfo, int N) {
    b_lincomb<FP>(hw_blk(), ba, coef, out, nbaby, nblk, count, ct0, nl, pinfo, N);
}

template <int KB>
__global__ void k_lincomb_wide(const u64 *__restrict__ in, u64 *__restrict__ out, const double *__restrict__ W,
                               const double *__restrict__ c0, int M, int K, int KT, int count, int nl,
                               const PrimeInfo *__restrict__ pinfo, int N) {
    b_lincomb_wide<KB>(hw_blk(), in, out, W, c0, M, K, KT, count, nl, pinfo, N);
}

__global__ void __launch_bounds__(256) k_lincomb_wide_mfma(const u64 *__restrict__ in, u64 *__restrict__ out,
                                                           const int8_t *__restrict__ W8,
                                                           const double *__restrict__ c0,
                                                           const int *__restrict__ corr, int M, int K, int count,
                                                           int nl, const PrimeInfo *__restrict__ pinfo, int N) {
    __shared__ __align__(16) unsigned char lds[8 * 32 * kWideRow];
    b_lincomb_wide_mfma(hw_blk(), in, out, W8, c0, corr, M, K, count, nl, pinfo, N, lds);
}

template <int PL, bool RAW, int STEPS>
__global__ void __launch_bounds__(kMfmaThreads) k_modup_mfma(const u64 *__restrict__ xc, u64 *__restrict__ mu,
                                                             const ModUpPlan *__restrict__ plans,
                                                             const int8_t *__restrict__ w8,
                                                             const double *__restrict__ corr, int plan_stride,
                                                             int plan0, const PrimeInfo *__restrict__ pinfo, int nl,
                                                             int next, int dnum, int nmod, int N) {
    __shared__ __align__(16) unsigned char lds[kMfmaPos * (32 * STEPS + 16)];
    b_modup_mfma<PL, RAW, STEPS>(hw_blk(), xc, mu, plans, w8, corr, plan_stride, plan0, pinfo, nl, next, dnum, nmod, N,
                                 lds);
}

inline dim3 grid3(int N, int y, int z) { return dim3((unsigned)(N / kT), (unsigned)y, (unsigned)z); }

}  // namespace

// ------------------------------------------------------------ launchers

void launch_tensor(const bc_ctx *c, const u64 *a, const u64 *b, const u64 *addend, u64 *out, int count, int bcount,
                   int nl, int na, int nb, int nc, hipStream_t st) {
    if (tl_rec) {
        tl_rec->add(addend ? kPkTensorAdd : kPkTensor, grid3(c->N, nl, count),
                    PaTensor{a, b, addend, out, bcount, nl, na, nb, addend ? nc : nl, c->pinfo, c->N});
        return;
    }
    ProfScope ps(c, kProfTensor, 8.0 * c->N * nl * (2.0 * count + 2.0 * bcount + (addend ? 2.0 * count : 0) + 3.0 * count),
                 st);
    if (addend)
        k_tensor<true><<<grid3(c->N, nl, count), kT, 0, st>>>(a, b, addend, out, bcount, nl, na, nb, nc, c->pinfo,
                                                             c->N);
    else
        k_tensor<false><<<grid3(c->N, nl, count), kT, 0, st>>>(a, b, nullptr, out, bcount, nl, na, nb, nl, c->pinfo,
                                                              c->N);
}
void launch_addsub(const bc_ctx *c, const u64 *a, const u64 *b, u64 *out, int count, int bcount, int nl, int na,
                   int nb, int ncomp, bool sub, hipStream_t st) {
    if (tl_rec) {
        tl_rec->add(kPkAddSub, grid3(c->N, nl, count),
                    PaAddSub{a, b, out, bcount, nl, na, nb, ncomp, sub ? 1 : 0, c->pinfo, c->N});
        return;
    }
    k_addsub<<<grid3(c->N, nl, count), kT, 0, st>>>(a, b, out, bcount, nl, na, nb, ncomp, sub ? 1 : 0, c->pinfo,
                                                    c->N);
}
static ScalarArg scalar_arg(const bc_ctx *c, int64_t v, int nl) {
    ScalarArg s{};
    for (int i = 0; i < nl; i++) {
        u64 q = c->mod[i];
        u64 r = v >= 0 ? (u64)v % q : (q - ((u64)(-v) % q)) % q;
        s.w[i][0] = r;
        s.w[i][1] = h_shoup(r, q);
    }
    return s;
}
void launch_mul_scalar(const bc_ctx *c, const u64 *a, u64 *out, int count, int nl, int ncomp, int64_t v, hipStream_t st) {
    if (tl_rec) {
        tl_rec->add(kPkMulScalar, grid3(c->N, nl, count), PaScalar{a, out, nl, ncomp, scalar_arg(c, v, nl), c->pinfo, c->N});
        return;
    }
    k_mul_scalar<<<grid3(c->N, nl, count), kT, 0, st>>>(a, out, nl, ncomp, scalar_arg(c, v, nl), c->pinfo, c->N);
}
void launch_add_const(const bc_ctx *c, const u64 *a, u64 *out, int count, int nl, int ncomp, int64_t v, hipStream_t st) {
    if (tl_rec) {
        tl_rec->add(kPkAddConst, grid3(c->N, nl, count), PaScalar{a, out, nl, ncomp, scalar_arg(c, v, nl), c->pinfo, c->N});
        return;
    }
    k_add_const<<<grid3(c->N, nl, count), kT, 0, st>>>(a, out, nl, ncomp, scalar_arg(c, v, nl), c->pinfo, c->N);
}
void launch_mul_monomial(const bc_ctx *c, const u64 *a, u64 *out, int count, int nl, int ncomp, int e, hipStream_t st) {
    BC_REQUIRE(e >= 0 && e < 2 * c->N, BC_ERR_ARG, "monomial exponent out of range");
    BC_REQUIRE(!tl_rec, BC_ERR_ARG, "the persistent executor does not run monomial products");
    k_mul_monomial<<<grid3(c->N, nl, count), kT, 0, st>>>(a, out, nl, ncomp, e, c->tw, c->pinfo, c->N, c->logN);
}
void launch_permute(const bc_ctx *c, const u64 *in, u64 *out, const u32 *perm, int count, int nl, int ncomp,
                    hipStream_t st, bool add0) {
    BC_REQUIRE(!add0 || in != out, BC_ERR_ARG, "permute-and-add runs out of place");
    k_permute<<<grid3(c->N, nl, count), kT, 0, st>>>(in, out, perm, nl, ncomp, c->N, c->pinfo, add0);
}
template <int PL, bool RAW, int STEPS>
static void modup_mfma_k(const bc_ctx *c, const ModUpMfma &T, const u64 *xc, u64 *mu, const ModUpPlan *plans, int count,
                         int level, int next, hipStream_t st) {
    const dim3 g((unsigned)((c->N >> PL) / kMfmaPos), 1, (unsigned)(count * c->dnum));
    k_modup_mfma<PL, RAW, STEPS><<<g, kMfmaThreads, 0, st>>>(xc, mu, plans, T.w8, T.corr, T.plan_stride,
                                                              level * c->dnum, c->pinfo, level + 1, next, c->dnum,
                                                              c->nmod, c->N);
}
template <int PL, bool RAW>
static void modup_mfma_r(const bc_ctx *c, const ModUpMfma &T, const u64 *xc, u64 *mu, const ModUpPlan *plans,
                         int count, int level, int next, hipStream_t st) {
    switch (T.kpad / 32) {
        case 1: return modup_mfma_k<PL, RAW, 1>(c, T, xc, mu, plans, count, level, next, st);
        case 2: return modup_mfma_k<PL, RAW, 2>(c, T, xc, mu, plans, count, level, next, st);
        case 3: return modup_mfma_k<PL, RAW, 3>(c, T, xc, mu, plans, count, level, next, st);
        case 4: return modup_mfma_k<PL, RAW, 4>(c, T, xc, mu, plans, count, level, next, st);
        case 5: return modup_mfma_k<PL, RAW, 5>(c, T, xc, mu, plans, count, level, next, st);
        case 6: return modup_mfma_k<PL, RAW, 6>(c, T, xc, mu, plans, count, level, next, st);
        case 7: return modup_mfma_k<PL, RAW, 7>(c, T, xc, mu, plans, count, level, next, st);
        case 8: return modup_mfma_k<PL, RAW, 8>(c, T, xc, mu, plans, count, level, next, st);
        default: throw Error(BC_ERR_ARG, "modulus raising on the matrix cores: digit too wide");
    }
}
template <int PL>
static void launch_modup_mfma(const bc_ctx *c, const ModUpMfma &T, const u64 *xc, u64 *mu, const ModUpPlan *plans,
                              int count, int level, int next, bool raw, hipStream_t st) {
    if (raw) modup_mfma_r<PL, true>(c, T, xc, mu, plans, count, level, next, st);
    else modup_mfma_r<PL, false>(c, T, xc, mu, plans, count, level, next, st);
}
template <bool FP, int PL, int MD>
static void modup_pl(const bc_ctx *c, const u64 *xc, u64 *mu, int count, int level, int next, bool raw,
                     hipStream_t st) {
    BC_REQUIRE(!raw || (FP && !tl_rec), BC_ERR_ARG, "reduced fp64 words: ordinary fp64 launches only");
    if (tl_rec) {
        static_assert(MD == (PL > 0 ? kFoldDigit : kMaxDigit), "the executor runs the launchers' digit bounds");
        BC_REQUIRE(FP, BC_ERR_ARG, "the persistent executor needs fp64 arithmetic");
        tl_rec->add(PL == 2 ? kPkModUp2 : PL == 1 ? kPkModUp1 : kPkModUp0, grid3(c->N >> PL, 1, count * c->dnum),
                    PaModUp{xc, mu, c->modup_f + (size_t)level * c->dnum, c->pinfo, level + 1, next, c->dnum, c->N});
        return;
    }
    const ModUpPlan *plans = (FP ? c->modup_f : c->modup) + (size_t)level * c->dnum;
    if constexpr (FP) {
        const ModUpMfma &T = c->modup_mfma[PL];
        if (c->mfma_modup && T.w8) {
            launch_modup_mfma<PL>(c, T, xc, mu, plans, count, level, next, raw, st);
            return;
        }
    }
    const dim3 g = grid3(c->N >> PL, 1, count * c->dnum);
    if (FP && raw) k_modup<FP, PL, MD, FP><<<g, kT, 0, st>>>(xc, mu, plans, c->pinfo, level + 1, next, c->dnum, c->N);
    else k_modup<FP, PL, MD><<<g, kT, 0, st>>>(xc, mu, plans, c->pinfo, level + 1, next, c->dnum, c->N);
}
template <bool FP>
static void modup_a(const bc_ctx *c, const u64 *xc, u64 *mu, int count, int level, int next, int pl, bool raw,
                    hipStream_t st) {
    if (pl == 2) modup_pl<FP, 2, kFoldDigit>(c, xc, mu, count, level, next, raw, st);
    else if (pl == 1) modup_pl<FP, 1, kFoldDigit>(c, xc, mu, count, level, next, raw, st);
    else modup_pl<FP, 0, kMaxDigit>(c, xc, mu, count, level, next, raw, st);
}
void launch_modup(const bc_ctx *c, const u64 *xc, u64 *mu, int count, int level, int next, int pl, hipStream_t st,
                  bool raw) {
    double limbs = 0;  // each digit's source limbs read, its new limbs written
    for (int j = 0; j < c->dnum; j++) {
        const ModUpPlan &p = c->h_modup[(size_t)level * c->dnum + j];
        if (p.nsrc) limbs += p.nsrc + p.ntgt;
    }
    ProfScope ps(c, kProfModUp, 8.0 * c->N * limbs * count, st);
    if (use_fp64(c)) modup_a<true>(c, xc, mu, count, level, next, pl, raw, st);
    else modup_a<false>(c, xc, mu, count, level, next, pl, raw, st);
}
void launch_ks_inner(const bc_ctx *c, const u64 *mu, const u64 *x, size_t x_ct_stride, const u64 *key, u64 *acc,
                     int count, int level, int next, int nact, hipStream_t st, bool raw) {
    BC_REQUIRE(!raw || (use_fp64(c) && !tl_rec), BC_ERR_ARG, "reduced fp64 words: ordinary fp64 launches only");
    // raised limbs of every active digit read, two accumulators written, the key read once
    ProfScope ps(c, kProfKsInner, 8.0 * c->N * next * ((double)count * (nact + 2) + 2.0 * nact), st);
    const dim3 g = grid3(c->N, next, (count + kKsCts - 1) / kKsCts);
    if (tl_rec) {
        BC_REQUIRE(use_fp64(c), BC_ERR_ARG, "the persistent executor needs fp64 arithmetic");
        tl_rec->add(kPkKsInner, g, PaKsInner{mu, x, x_ct_stride, key, acc, level, c->nQ, c->nmod, next, nact, c->dnum,
                                             c->alpha, count, c->pinfo, c->N});
        return;
    }
    if (use_fp64(c) && raw)
        k_ks_inner<true, true><<<g, kT, 0, st>>>(mu, x, x_ct_stride, key, acc, level, c->nQ, c->nmod, next, nact,
                                                 c->dnum, c->alpha, count, c->pinfo, c->N);
    else if (use_fp64(c))
        k_ks_inner<true><<<g, kT, 0, st>>>(mu, x, x_ct_stride, key, acc, level, c->nQ, c->nmod, next, nact, c->dnum,
                                           c->alpha, count, c->pinfo, c->N);
    else
        k_ks_inner<false><<<g, kT, 0, st>>>(mu, x, x_ct_stride, key, acc, level, c->nQ, c->nmod, next, nact, c->dnum,
                                            c->alpha, count, c->pinfo, c->N);
}
template <bool FP, int PL>
static void moddown_pl(const bc_ctx *c, const u64 *acc, u64 *th, int count, int level, int next, bool scaled,
                       hipStream_t st) {
    const ModDownPlan *md = FP ? c->moddown_f : c->moddown;
    if (tl_rec) {
        BC_REQUIRE(FP && !scaled, BC_ERR_ARG, "the persistent executor needs fp64 arithmetic, unscaled lowering");
        tl_rec->add(PL == 2 ? kPkModDown2 : PL == 1 ? kPkModDown1 : kPkModDown0, grid3(c->N >> PL, 1, count * 2),
                    PaModDown{acc, th, md, c->pinfo, level, c->nQ, c->nP, next, c->N});
        return;
    }
    const dim3 g = grid3(c->N >> PL, 1, count * 2);
    if (scaled) k_moddown<FP, PL, true><<<g, kT, 0, st>>>(acc, th, md, c->pinfo, level, c->nQ, c->nP, next, c->N);
    else k_moddown<FP, PL><<<g, kT, 0, st>>>(acc, th, md, c->pinfo, level, c->nQ, c->nP, next, c->N);
}
template <bool FP>
static void moddown_a(const bc_ctx *c, const u64 *acc, u64 *th, int count, int level, int next, int pl,
                      bool scaled, hipStream_t st) {
    if (pl == 2) moddown_pl<FP, 2>(c, acc, th, count, level, next, scaled, st);
    else if (pl == 1) moddown_pl<FP, 1>(c, acc, th, count, level, next, scaled, st);
    else moddown_pl<FP, 0>(c, acc, th, count, level, next, scaled, st);
}
void launch_moddown(const bc_ctx *c, const u64 *acc, u64 *th, int count, int level, int next, int pl, hipStream_t st,
                    bool scaled) {
    BC_REQUIRE(pl == 0 || (c->nP <= kFoldDigit), BC_ERR_PARAM, "modulus lowering: too many special primes to fold");
    if (use_fp64(c)) moddown_a<true>(c, acc, th, count, level, next, pl, scaled, st);
    else moddown_a<false>(c, acc, th, count, level, next, pl, scaled, st);
}
void launch_ks_combine(const bc_ctx *c, const u64 *base0, const u64 *base1, size_t base_ct_stride, const u64 *acc,
                       const u64 *th, u64 *out, size_t out_ct_stride, int count, int level, int next, hipStream_t st) {
    if (tl_rec) {
        tl_rec->add(kPkKsCombine, grid3(c->N, level + 1, count),
                    PaKsCombine{base0, base1, base_ct_stride, acc, th, out, out_ct_stride, c->moddown, c->pinfo,
                                level + 1, next, c->N});
        return;
    }
    k_ks_combine<<<grid3(c->N, level + 1, count), kT, 0, st>>>(base0, base1, base_ct_stride, acc, th, out,
                                                               out_ct_stride, c->moddown, c->pinfo, level + 1, next,
                                                               c->N);
}
template <bool FP, int PL>
static void ms_fbc_pl(const bc_ctx *c, const u64 *top, u64 *R, int count, int level, hipStream_t st) {
    k_ms_fbc<FP, PL><<<grid3(c->N >> PL, 1, count * 2), kT, 0, st>>>(top, R, (FP ? c->modsw_f : c->modsw) + level,
                                                                    c->pinfo, level, c->N);
}
template <bool FP>
static void ms_fbc_a(const bc_ctx *c, const u64 *top, u64 *R, int count, int level, int pl, hipStream_t st) {
    if (pl == 2) ms_fbc_pl<FP, 2>(c, top, R, count, level, st);
    else if (pl == 1) ms_fbc_pl<FP, 1>(c, top, R, count, level, st);
    else ms_fbc_pl<FP, 0>(c, top, R, count, level, st);
}
void launch_ms_fbc(const bc_ctx *c, const u64 *top, u64 *R, int count, int level, int pl, hipStream_t st) {
    if (use_fp64(c)) ms_fbc_a<true>(c, top, R, count, level, pl, st);
    else ms_fbc_a<false>(c, top, R, count, level, pl, st);
}
template <bool FP, int PL, int MD>
static void relin_ms_fbc_pl(const bc_ctx *c, const u64 *acc, const u64 *d, size_t d_ct_stride, u64 *E, int count,
                            int level, int next, bool raw, hipStream_t st) {
    BC_REQUIRE(!raw || (FP && !tl_rec), BC_ERR_ARG, "reduced fp64 words: ordinary fp64 launches only");
    if (tl_rec) {
        static_assert(MD == (PL > 0 ? kFoldDigit : kMaxDigit), "the executor runs the launchers' digit bounds");
        BC_REQUIRE(FP, BC_ERR_ARG, "the persistent executor needs fp64 arithmetic");
        tl_rec->add(PL == 2 ? kPkRelinMs2 : PL == 1 ? kPkRelinMs1 : kPkRelinMs0, grid3(c->N >> PL, 1, count * 2),
                    PaRelinMs{acc, d, d_ct_stride, E, c->moddown_f, c->modsw_f + level, c->pinfo, level, c->nQ, c->nP,
                              next, c->N});
        return;
    }
    const dim3 g = grid3(c->N >> PL, 1, count * 2);
    const ModDownPlan *md = FP ? c->moddown_f : c->moddown;
    const ModSwitchPlan *ms = (FP ? c->modsw_f : c->modsw) + level;
    if (FP && raw)
        k_relin_ms_fbc<FP, PL, MD, FP><<<g, kT, 0, st>>>(acc, d, d_ct_stride, E, md, ms, c->pinfo, level, c->nQ, c->nP,
                                                        next, c->N);
    else
        k_relin_ms_fbc<FP, PL, MD><<<g, kT, 0, st>>>(acc, d, d_ct_stride, E, md, ms, c->pinfo, level, c->nQ, c->nP,
                                                    next, c->N);
}
template <bool FP>
static void relin_ms_fbc_a(const bc_ctx *c, const u64 *acc, const u64 *d, size_t d_ct_stride, u64 *E, int count,
                           int level, int next, int pl, bool raw, hipStream_t st) {
    if (pl == 2) relin_ms_fbc_pl<FP, 2, kFoldDigit>(c, acc, d, d_ct_stride, E, count, level, next, raw, st);
    else if (pl == 1) relin_ms_fbc_pl<FP, 1, kFoldDigit>(c, acc, d, d_ct_stride, E, count, level, next, raw, st);
    else relin_ms_fbc_pl<FP, 0, kMaxDigit>(c, acc, d, d_ct_stride, E, count, level, next, raw, st);
}
void launch_relin_ms_fbc(const bc_ctx *c, const u64 *acc, const u64 *d, size_t d_ct_stride, u64 *E, int count,
                         int level, int next, int pl, hipStream_t st, bool raw) {
    // per component: the special and top accumulator limbs and d's top limb read, `level` limbs written
    ProfScope ps(c, kProfRelinMs, 8.0 * c->N * 2.0 * count * (c->nP + 2 + level), st);
    if (use_fp64(c)) relin_ms_fbc_a<true>(c, acc, d, d_ct_stride, E, count, level, next, pl, raw, st);
    else relin_ms_fbc_a<false>(c, acc, d, d_ct_stride, E, count, level, next, pl, raw, st);
}
void launch_relin_ms_combine(const bc_ctx *c, const u64 *d, size_t d_ct_stride, const u64 *acc, const u64 *E, u64 *out,
                             int count, int level, int next, hipStream_t st) {
    PairArg pa{};
    const u64 ql = c->mod[level];
    for (int i = 0; i < level; i++) {
        const u64 q = c->mod[i];
        u64 P = 1;
        for (int t = 0; t < c->nP; t++) P = h_mulmod(P, c->mod[c->nQ + t] % q, q);
        const u64 qlinv = h_invmod(ql % q, q), pq = h_mulmod(h_invmod(P, q), qlinv, q);
        pa.w[i][0] = qlinv;
        pa.w[i][1] = h_shoup(qlinv, q);
        pa.w[i][2] = pq;
        pa.w[i][3] = h_shoup(pq, q);
    }
    k_relin_ms_combine<<<grid3(c->N, level, count), kT, 0, st>>>(d, d_ct_stride, acc, E, out, pa, c->pinfo, level,
                                                                 next, c->N);
}
void launch_ms_combine(const bc_ctx *c, const u64 *in, const u64 *R, u64 *out, int count, int level, hipStream_t st) {
    k_ms_combine<<<grid3(c->N, level, count), kT, 0, st>>>(in, R, out, c->modsw + level, c->pinfo, level, c->N);
}
void launch_words_mod(const bc_ctx *c, const u64 *w, u64 *out, const int16_t *primes, int npoly, int nlimb,
                      hipStream_t st) {
    k_words_mod<<<grid3(c->N, nlimb, npoly), kT, 0, st>>>(w, out, primes, c->pinfo, nlimb, c->N);
}
void launch_lift_small(const bc_ctx *c, const int32_t *v32, const int8_t *v8, size_t vstride, const uint32_t *add,
                       u64 *out, const int16_t *primes, int npoly, int nlimb, bool use_p, hipStream_t st) {
    k_lift_small<<<grid3(c->N, nlimb, npoly), kT, 0, st>>>(v32, v8, vstride, add, out, primes, c->pinfo, nlimb,
                                                          use_p ? 1 : 0, c->N);
}
void launch_keypair(const bc_ctx *c, const u64 *A, const u64 *E, const u64 *S, const u64 *S2, const u64 *f, u64 *k0,
                    u64 *k1, int nlimb, hipStream_t st) {
    FArg fa{};
    for (int i = 0; i < nlimb; i++) fa.f[i] = f ? f[i] : 0;
    k_keypair<<<grid3(c->N, nlimb, 1), kT, 0, st>>>(A, E, S, S2, fa, k0, k1, c->pinfo, c->N);
}
void launch_pmul(const bc_ctx *c, const u64 *a, const u64 *b, u64 *out, int nlimb, hipStream_t st) {
    k_pmul<<<grid3(c->N, nlimb, 1), kT, 0, st>>>(a, b, out, c->pinfo, c->N);
}
void launch_enc_combine(const bc_ctx *c, const u64 *pk, const u64 *U, const u64 *E0, const u64 *E1, u64 *out, int count,
                        hipStream_t st) {
    k_enc_combine<<<grid3(c->N, c->nQ, count), kT, 0, st>>>(pk, U, E0, E1, out, c->nQ, c->pinfo, c->N);
}
void launch_dec_inner(const bc_ctx *c, const u64 *ct, const u64 *s, u64 *d, int count, int nl, int ncomp, hipStream_t st) {
    k_dec_inner<<<grid3(c->N, nl, count), kT, 0, st>>>(ct, s, d, nl, ncomp, c->pinfo, c->N);
}
void launch_lincomb(const bc_ctx *c, const u64 *const *babies, const int *nlb, const int *pos, const u64 *coef,
                    u64 *out, int nbaby, int nblk, int count, int ct0, int nlaunch, int nl, hipStream_t st) {
    BC_REQUIRE(nbaby <= 16 && nblk <= 64, BC_ERR_PARAM, "schedule too large");
    BabyArg ba{};
    for (int k = 0; k < nbaby; k++) {
        BC_REQUIRE(nlb[k] >= nl, BC_ERR_LEVEL, "a baby step below the blocks' level");
        ba.baby[k] = babies[k];
        ba.nlb[k] = nlb[k];
    }
    for (int t = 0; t < nblk; t++) ba.pos[t] = pos[t];
    if (tl_rec) {
        tl_rec->add(lincomb_small(c) ? kPkLincombFp : kPkLincombInt, grid3(c->N, nl, 2 * nlaunch),
                    PaLincomb{ba, coef, out, nbaby, nblk, count, ct0, nl, c->pinfo, c->N});
        return;
    }
    ProfScope ps(c, kProfLincomb, 8.0 * c->N * 2.0 * nl * nlaunch * (nbaby + nblk), st);
    if (lincomb_small(c))
        k_lincomb<true><<<grid3(c->N, nl, 2 * nlaunch), kT, 0, st>>>(ba, coef, out, nbaby, nblk, count, ct0, nl,
                                                                    c->pinfo, c->N);
    else
        k_lincomb<false><<<grid3(c->N, nl, 2 * nlaunch), kT, 0, st>>>(ba, coef, out, nbaby, nblk, count, ct0, nl, c->pinfo,
                                                                 c->N);
}
int lincomb_wide_tile(int K) { return K >= 16 ? 16 : K >= 8 ? 8 : 1; }
void launch_lincomb_wide(const bc_ctx *c, const u64 *in, u64 *out, const double *W, const double *c0, int M, int K,
                         int count, int nl, hipStream_t st) {
    BC_REQUIRE(use_fp64(c), BC_ERR_PARAM, "wide linear combinations need primes below 2^50");
    BC_REQUIRE(!tl_rec, BC_ERR_ARG, "the persistent executor does not run wide linear combinations");
    BC_REQUIRE(M >= 1 && M <= 4096 && K >= 1, BC_ERR_ARG, "wide linear combination: bad shape");
    const int KB = lincomb_wide_tile(K), KT = (K + KB - 1) / KB;
    ProfScope ps(c, kProfLincomb, 8.0 * c->N * 2.0 * nl * count * (M + K), st);
    const dim3 g((unsigned)(KT * (c->N / kT)), (unsigned)nl, (unsigned)(2 * count));
    if (KB == 16) k_lincomb_wide<16><<<g, kT, 0, st>>>(in, out, W, c0, M, K, KT, count, nl, c->pinfo, c->N);
    else if (KB == 8) k_lincomb_wide<8><<<g, kT, 0, st>>>(in, out, W, c0, M, K, KT, count, nl, c->pinfo, c->N);
    else k_lincomb_wide<1><<<g, kT, 0, st>>>(in, out, W, c0, M, K, KT, count, nl, c->pinfo, c->N);
}
void launch_lincomb_wide_mfma(const bc_ctx *c, const u64 *in, u64 *out, const int8_t *W8, const double *c0,
                              const int *corr, int M, int K, int count, int nl, hipStream_t st) {
    BC_REQUIRE(use_fp64(c), BC_ERR_PARAM, "wide linear combinations need primes below 2^50");
    BC_REQUIRE(!tl_rec, BC_ERR_ARG, "the persistent executor does not run wide linear combinations");
    BC_REQUIRE(M >= 1 && M <= kWideMfmaM && K >= 1 && K <= kWideMfmaK && c->N % 32 == 0, BC_ERR_ARG,
               "wide linear combination on the matrix cores: bad shape");
    ProfScope ps(c, kProfLincomb, 8.0 * c->N * 2.0 * nl * count * (M + K), st);
    const dim3 g((unsigned)(c->N / 32), (unsigned)nl, (unsigned)(2 * count));
    k_lincomb_wide_mfma<<<g, 256, 0, st>>>(in, out, W8, c0, corr, M, K, count, nl, c->pinfo, c->N);
}
void launch_crt_decode(const bc_ctx *c, const u64 *d, uint32_t *out, int count, int nl, hipStream_t st) {
    k_crt_decode<<<grid3(c->N, 1, count), kT, 0, st>>>(d, out, c->garner, c->pinfo, nl, c->p, c->N);
}

// ------------------------------------------------- allocation-free workspace
// Workspace of the allocation-free multiplication: a fixed device array of
// kScratchBytes (every GPU the library runs on holds its own copy until the
// process ends).  In host code the array's name only stands for the symbol:
// its device address is looked up once per device, with that device current,
// and only that address is ever handed to kernels or copies.
static __device__ __align__(256) u64 scratch[kScratchBytes / sizeof(u64)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_addr[kMaxDevices];
}  // namespace

void *scratch_lookup(int device) {
    BC_REQUIRE(device >= 0 && device < kMaxDevices, BC_ERR_HIP, "device index out of range");
    std::lock_guard<std::mutex> g(scratch_mu);
    if (!scratch_addr[device]) {
        void *ptr = nullptr;
        BC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        BC_REQUIRE(ptr, BC_ERR_HIP, "no device address for the allocation-free workspace");
        scratch_addr[device] = ptr;
    }
    return scratch_addr[device];
}

}  // namespace bc
