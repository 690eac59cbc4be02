// kernels.h -- host launchers of the element-wise and conversion kernels.
#pragma once

#include "bc_internal.h"

namespace bc {

void build_context(bc_ctx *c, const bc_params &prm);
void build_context_moduli(bc_ctx *c, const bc_params &prm, std::vector<u64> mod);
// the `count` largest primes below 2^bits that are 1 mod step, decreasing
std::vector<u64> primes_one_mod(u64 step, int bits, int count);

// Size of the fixed device workspace of the allocation-free multiplication
// (one array per GPU, kept until the process ends).
constexpr size_t kScratchBytes = (size_t)64 << 20;
// Device address of that workspace on `device`, which must be the current
// device; looked up on the first call per device, then cached.
void *scratch_lookup(int device);

// The output has nl limbs per component; na, nb, nc (>= nl) are the limbs
// per component the operands are stored with (their lowest nl are read).
// addend: null, or [count][2][nc][N] added to the first two components.
void launch_tensor(const bc_ctx *c, const u64 *a, const u64 *b, const u64 *addend, u64 *out, int count, int bcount,
                   int nl, int na, int nb, int nc, hipStream_t st);
void launch_addsub(const bc_ctx *c, const u64 *a, const u64 *b, u64 *out, int count, int bcount, int nl, int na,
                   int nb, int ncomp, bool sub, hipStream_t st);
void launch_mul_scalar(const bc_ctx *c, const u64 *a, u64 *out, int count, int nl, int ncomp, int64_t v, hipStream_t st);
void launch_add_const(const bc_ctx *c, const u64 *a, u64 *out, int count, int nl, int ncomp, int64_t v, hipStream_t st);
// out = a x^e (0 <= e < 2N) on count batches of nl limbs x ncomp components (NTT domain; in place allowed)
void launch_mul_monomial(const bc_ctx *c, const u64 *a, u64 *out, int count, int nl, int ncomp, int e, hipStream_t st);
// add0: component 0 gets the input's own component 0 added (in != out)
void launch_permute(const bc_ctx *c, const u64 *in, u64 *out, const u32 *perm, int count, int nl, int ncomp,
                    hipStream_t st, bool add0 = false);
// `pl`: the first pl forward stages of the transforms that follow are applied
// to the outputs (ntt_parts_log(c), or 0)
// raw: the input and the new limbs as reduced fp64 patterns (fp64 arithmetic,
// ordinary launches; see LimbSet::raw_in)
void launch_modup(const bc_ctx *c, const u64 *xc, u64 *mu, int count, int level, int next, int pl, hipStream_t st,
                  bool raw = false);
// raw: mu's raised limbs as reduced fp64 patterns
void launch_ks_inner(const bc_ctx *c, const u64 *mu, const u64 *x, size_t x_ct_stride, const u64 *key, u64 *acc,
                     int count, int level, int next, int nact, hipStream_t st, bool raw = false);
// pl > 0: the special limbs come from part-limb inverse transforms (their
// last pl stages are applied here) and TH goes to part-limb forward ones
// (their first pl stages are applied here)
// scaled: TH p P^-1 instead of TH (for the rotation's fused key-switch combine)
void launch_moddown(const bc_ctx *c, const u64 *acc, u64 *th, int count, int level, int next, int pl, hipStream_t st,
                    bool scaled = false);
void launch_ks_combine(const bc_ctx *c, const u64 *base0, const u64 *base1, size_t base_ct_stride, const u64 *acc,
                       const u64 *th, u64 *out, size_t out_ct_stride, int count, int level, int next, hipStream_t st);
void launch_ms_fbc(const bc_ctx *c, const u64 *top, u64 *R, int count, int level, int pl, hipStream_t st);
// raw: the coefficient-domain inputs and E as reduced fp64 patterns
void launch_relin_ms_fbc(const bc_ctx *c, const u64 *acc, const u64 *d, size_t d_ct_stride, u64 *E, int count,
                         int level, int next, int pl, hipStream_t st, bool raw = false);
void launch_relin_ms_combine(const bc_ctx *c, const u64 *d, size_t d_ct_stride, const u64 *acc, const u64 *E, u64 *out,
                             int count, int level, int next, hipStream_t st);
void launch_ms_combine(const bc_ctx *c, const u64 *in, const u64 *R, u64 *out, int count, int level, hipStream_t st);
void launch_words_mod(const bc_ctx *c, const u64 *w, u64 *out, const int16_t *primes, int npoly, int nlimb,
                      hipStream_t st);
void launch_lift_small(const bc_ctx *c, const int32_t *v32, const int8_t *v8, size_t vstride, const uint32_t *add,
                       u64 *out, const int16_t *primes, int npoly, int nlimb, bool use_p, hipStream_t st);
void launch_keypair(const bc_ctx *c, const u64 *A, const u64 *E, const u64 *S, const u64 *S2, const u64 *f, u64 *k0,
                    u64 *k1, int nlimb, hipStream_t st);
void launch_pmul(const bc_ctx *c, const u64 *a, const u64 *b, u64 *out, int nlimb, hipStream_t st);
void launch_enc_combine(const bc_ctx *c, const u64 *pk, const u64 *U, const u64 *E0, const u64 *E1, u64 *out, int count,
                        hipStream_t st);
void launch_dec_inner(const bc_ctx *c, const u64 *ct, const u64 *s, u64 *d, int count, int nl, int ncomp, hipStream_t st);
void launch_lincomb(const bc_ctx *c, const u64 *const *babies, const int *nlb, const int *pos, const u64 *coef,
                    u64 *out, int nbaby, int nblk, int count, int ct0, int nlaunch, int nl, hipStream_t st);
// out[k] = sum_m W[k][m] in[m] (+ c0[k] on component 0), k < K: in is M
// compact blocks of `count` ciphertexts at nl limbs, out K blocks; W is
// [KT tile][M] doubles (KT = ceil(K / tile), rows past K zero), |W| <= 2^8,
// M <= 4096; c0 [KT tile] doubles.  fp64 contexts only.
int lincomb_wide_tile(int K);
void launch_lincomb_wide(const bc_ctx *c, const u64 *in, u64 *out, const double *W, const double *c0, int M, int K,
                         int count, int nl, hipStream_t st);
// The same on the matrix cores (exact split-int8 products): W8 int8 [128][256]
// with the weights equal to 128 zeroed and listed in corr (offsets [K + 1],
// then input indices); M <= 256, K <= 128.
void launch_lincomb_wide_mfma(const bc_ctx *c, const u64 *in, u64 *out, const int8_t *W8, const double *c0,
                              const int *corr, int M, int K, int count, int nl, hipStream_t st);
void launch_crt_decode(const bc_ctx *c, const u64 *d, uint32_t *out, int count, int nl, hipStream_t st);

}  // namespace bc
