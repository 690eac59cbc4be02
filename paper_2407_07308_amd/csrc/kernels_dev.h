// kernels_dev.h -- device bodies of the element-wise, base-conversion and
// key-switching kernels.
//
// Each body computes one workgroup's share of its kernel from the block
// coordinates it is given (VBlk): the hardware's when a kernel of its own
// runs it, a virtual block's when the persistent executor does.  Every
// ciphertext limb is a contiguous run of N uint64 residues; a batch is
// [count][ncomp][nlimb][N]; x covers the N coefficients of a limb (256 per
// workgroup), y the limb, z the ciphertext of the batch.
#pragma once

#include <type_traits>

#include "bc_internal.h"

namespace bc {

namespace {

constexpr int kT = 256;

__device__ __forceinline__ int ext_prime(int e, int level, int nQ) { return e <= level ? e : nQ + (e - level - 1); }


// ACC[ct][c][e] = sum_j MU[ct][j][e] * K_j,c[prime(e)]   (NTT domain), where
// digit j's own limbs (e in [j alpha, (j+1) alpha)) are X's limbs themselves.
// A thread takes kKsCts consecutive ciphertexts: each key word is read once
// for all of them, and every load is issued before the arithmetic.
constexpr int kKsCts = 8;


// (a0 b0, a0 b1 + a1 b0, a1 b1), plus (c0, c1) on the first two components
// when an addend c is given (a multiply-accumulate's sum before relinearising).
// The output has nl limbs; each operand is read at its own limb count (na,
// nb, nc >= nl): an operand above the output's level contributes its lowest
// nl limbs (level alignment by dropping primes, without a copy).  When b is
// broadcast (bcount < count, ciphertext ct uses b[ct % bcount]) the grid runs
// the count / bcount products that share a b ciphertext back to back, so
// its limbs come from the cache after the first.
template <bool ADD>
__device__ __forceinline__ void b_tensor(const VBlk &VB, const u64 *__restrict__ a, const u64 *__restrict__ b, const u64 *__restrict__ c,
                         u64 *__restrict__ out, int bcount, int nl, int na, int nb, int nc,
                         const PrimeInfo *__restrict__ pinfo, int N) {
    const int rep = VB.gz / bcount;  // products per b ciphertext
    const int n = VB.x * kT + threadIdx.x, i = VB.y;
    const int ct = (int)(VB.z % rep) * bcount + (int)(VB.z / rep);
    const size_t L = (size_t)nl * N, La = (size_t)na * N, Lb = (size_t)nb * N;
    const u64 *A = a + (size_t)ct * 2 * La + (size_t)i * N + n;
    const u64 *B = b + (size_t)(ct % bcount) * 2 * Lb + (size_t)i * N + n;
    u64 *O = out + (size_t)ct * 3 * L + (size_t)i * N + n;
    const Barrett br = pinfo[i].br;
    u64 a0 = A[0], a1 = A[La], b0 = B[0], b1 = B[Lb];
    u64 d0 = mul_mod(a0, b0, br), d1 = add_mod(mul_mod(a0, b1, br), mul_mod(a1, b0, br), br.q);
    if constexpr (ADD) {
        const size_t Lc = (size_t)nc * N;
        const u64 *C = c + (size_t)ct * 2 * Lc + (size_t)i * N + n;
        d0 = add_mod(d0, C[0], br.q);
        d1 = add_mod(d1, C[Lc], br.q);
    }
    O[0] = d0;
    O[L] = d1;
    O[2 * L] = mul_mod(a1, b1, br);
}

// out = a + sgn * b on ncomp components (sgn = +1 / -1); out has nl limbs,
// a and b are read at their own limb counts (na, nb >= nl)
__device__ __forceinline__ void b_addsub(const VBlk &VB, const u64 *__restrict__ a, const u64 *__restrict__ b, u64 *__restrict__ out, int bcount,
                         int nl, int na, int nb, int ncomp, int sub, const PrimeInfo *__restrict__ pinfo, int N) {
    const int n = VB.x * kT + threadIdx.x, i = VB.y, ct = VB.z;
    const size_t L = (size_t)nl * N, La = (size_t)na * N, Lb = (size_t)nb * N;
    const u64 q = pinfo[i].q;
    for (int c = 0; c < ncomp; c++) {
        const size_t off = (size_t)i * N + n;
        u64 x = a[(size_t)ct * ncomp * La + c * La + off], y = b[(size_t)(ct % bcount) * ncomp * Lb + c * Lb + off];
        out[(size_t)ct * ncomp * L + c * L + off] = sub ? sub_mod(x, y, q) : add_mod(x, y, q);
    }
}

__device__ __forceinline__ void b_mul_scalar(const VBlk &VB, const u64 *__restrict__ a, u64 *__restrict__ out, int nl, int ncomp, const ScalarArg &s,
                             const PrimeInfo *__restrict__ pinfo, int N) {
    const int n = VB.x * kT + threadIdx.x, i = VB.y, ct = VB.z;
    const size_t L = (size_t)nl * N;
    const u64 q = pinfo[i].q;
    for (int c = 0; c < ncomp; c++) {
        size_t off = (size_t)ct * ncomp * L + (size_t)c * L + (size_t)i * N + n;
        out[off] = shoup(a[off], s.w[i][0], s.w[i][1], q);
    }
}

// multiplication by the monomial x^e, 0 <= e < 2N: position r of a limb holds
// the evaluation at psi^(2 brv(r) + 1), where x^e is psi^(e (2 brv(r) + 1));
// psi^x for x < N is the table word W[brv(x)], and psi^(x + N) = -psi^x
__device__ __forceinline__ void b_mul_monomial(const VBlk &VB, const u64 *__restrict__ a, u64 *__restrict__ out, int nl,
                                               int ncomp, int e, const u64 *__restrict__ tw,
                                               const PrimeInfo *__restrict__ pinfo, int N, int logN) {
    const int n = VB.x * kT + threadIdx.x, i = VB.y, ct = VB.z;
    const size_t L = (size_t)nl * N;
    const u32 ev = 2u * (__brev((u32)n) >> (32 - logN)) + 1u;
    const u32 x = (u32)(((u64)e * ev) & (2u * (u64)N - 1));
    const bool neg = x >= (u32)N;
    const u32 r = __brev(neg ? x - (u32)N : x) >> (32 - logN);
    const u64 *W = tw + (size_t)i * 4 * N;
    const u64 w = W[r], wp = W[N + r], q = pinfo[i].q;
    for (int c = 0; c < ncomp; c++) {
        const size_t off = (size_t)ct * ncomp * L + (size_t)c * L + (size_t)i * N + n;
        const u64 v = shoup(a[off], w, wp, q);
        out[off] = neg && v ? q - v : v;
    }
}

// constant polynomial c: every evaluation of component 0 gains c mod q_i
__device__ __forceinline__ void b_add_const(const VBlk &VB, const u64 *__restrict__ a, u64 *__restrict__ out, int nl, int ncomp, const ScalarArg &s,
                            const PrimeInfo *__restrict__ pinfo, int N) {
    const int n = VB.x * kT + threadIdx.x, i = VB.y, ct = VB.z;
    const size_t L = (size_t)nl * N;
    const u64 q = pinfo[i].q;
    for (int c = 0; c < ncomp; c++) {
        size_t off = (size_t)ct * ncomp * L + (size_t)c * L + (size_t)i * N + n;
        u64 x = a[off];
        out[off] = c == 0 ? add_mod(x, s.w[i][0], q) : x;
    }
}

// out[ct][c][i][r] = in[ct][c][i][perm[r]]  (+ in[ct][0][i][r] on component 0
// when add0: the automorphism's component 0 with the input's own added, the
// base of a rotate-and-add's key switch)
__device__ __forceinline__ void b_permute(const VBlk &VB, const u64 *__restrict__ in, u64 *__restrict__ out, const u32 *__restrict__ perm, int nl,
                          int ncomp, int N, const PrimeInfo *__restrict__ pinfo = nullptr, bool add0 = false) {
    const int n = VB.x * kT + threadIdx.x, i = VB.y, ct = VB.z;
    const size_t L = (size_t)nl * N;
    const u32 src = perm[n];
    for (int c = 0; c < ncomp; c++) {
        size_t base = (size_t)ct * ncomp * L + (size_t)c * L + (size_t)i * N;
        const u64 x = in[base + src];
        out[base + n] = c == 0 && add0 ? add_mod(x, in[base + n], pinfo[i].q) : x;
    }
}

// Fast base conversion of digit j (z-grid = ct * dnum + j):
// y_i = [x_i Qhat_i^-1]_{q_i}, u_t = sum_i y_i Qhat_i mod q_t.
// With PL > 0 a thread takes the 2^PL words n + v N/2^PL of each limb: it
// applies the last PL stages of the part-limb inverse transform that made xc
// to its inputs (unfold_int / unfold_fp) and the first PL forward stages of
// the new limbs' transforms to its outputs (fold_int / fold_fp).  MD bounds
// the digit size at compile time.
// RAW (fp64 only): the input and the new limbs are reduced fp64 patterns
// (|x| <= q/2) instead of canonical words.
template <bool FP, int PL = 0, int MD = kMaxDigit, bool RAW = false>
__device__ __forceinline__ void b_modup(const VBlk &VB, const u64 *__restrict__ xc, u64 *__restrict__ mu, const ModUpPlan *__restrict__ plans,
                        const PrimeInfo *__restrict__ pinfo, int nl, int next, int dnum, int N) {
    constexpr int NV = 1 << PL;
    const int n = VB.x * kT + threadIdx.x, Q = N >> PL;
    const int ct = VB.z / dnum, j = VB.z - ct * dnum;
    const ModUpPlan &pl = plans[j];
    if (pl.nsrc == 0) return;
    u64 *out = mu + ((size_t)ct * dnum + j) * next * N + n;
    const u64 *in = xc + (size_t)ct * nl * N + n;
    if constexpr (!FP) {
        // fully unrolled over the compile-time bound so y[] stays in registers
        u64 y[NV][MD];
#pragma unroll
        for (int s = 0; s < MD; s++) {
            if (s >= pl.nsrc) break;
            const int i = pl.src_lo + s;
            u64 x[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) x[v] = in[(size_t)i * N + v * Q];
            if constexpr (PL > 0) unfold_int<PL>(x, pinfo[i]);
#pragma unroll
            for (int v = 0; v < NV; v++) y[v][s] = shoup(x[v], pl.qhinv[s][0], pl.qhinv[s][1], pinfo[i].q);
        }
        for (int t = 0; t < pl.ntgt; t++) {
            const PrimeInfo &pt = pinfo[pl.tgt_prime[t]];
            u64 acc[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) {
                acc[v] = 0;
#pragma unroll
                for (int s = 0; s < MD; s++) {
                    if (s >= pl.nsrc) break;
                    acc[v] = add_mod(acc[v], shoup(y[v][s], pl.qhat[t][s][0], pl.qhat[t][s][1], pt.q), pt.q);
                }
            }
            if constexpr (PL > 0) fold_int<PL>(acc, pt);
#pragma unroll
            for (int v = 0; v < NV; v++) out[(size_t)pl.tgt_e[t] * N + v * Q] = acc[v];
        }
    } else {
#pragma clang fp contract(off)
        // y_s canonical in [0, q_s); each product below 0.75 q_t in magnitude,
        // so eight of them sum exactly before a reduction
        double y[NV][MD];
#pragma unroll
        for (int s = 0; s < MD; s++) {
            if (s >= pl.nsrc) break;
            const PrimeInfo &pi = pinfo[pl.src_lo + s];
            double x[NV];
#pragma unroll
            for (int v = 0; v < NV; v++)
                x[v] = RAW ? f_raw_load(in[(size_t)(pl.src_lo + s) * N + v * Q]) : f_load(in[(size_t)(pl.src_lo + s) * N + v * Q]);
            if constexpr (PL > 0) unfold_fp<PL, false>(x, pi);  // |x| < 1.5 q: fine for the product
#pragma unroll
            for (int v = 0; v < NV; v++) y[v][s] = f_canon(f_mulmod(x[v], fpair(pl.qhinv[s]), pi.qd), pi.qd, pi.qinv);
        }
        for (int t = 0; t < pl.ntgt; t++) {
            const PrimeInfo &pt = pinfo[pl.tgt_prime[t]];
            double acc[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) {
                acc[v] = 0.0;
#pragma unroll
                for (int s = 0; s < MD; s++) {
                    if (s >= pl.nsrc) break;
                    acc[v] += f_mulmod(y[v][s], fpair(pl.qhat[t][s]), pt.qd);
                    if ((s & 7) == 7) acc[v] = f_reduce(acc[v], pt.qd, pt.qinv);
                }
                // the fold takes |x| < 1.6 q and returns canonical (reduced) words
                acc[v] = PL > 0 || RAW ? f_reduce(acc[v], pt.qd, pt.qinv) : f_canon(acc[v], pt.qd, pt.qinv);
            }
            if constexpr (PL > 0) fold_fp<PL, !RAW>(acc, pt);
#pragma unroll
            for (int v = 0; v < NV; v++) out[(size_t)pl.tgt_e[t] * N + v * Q] = RAW ? f_raw_bits(acc[v]) : f_bits(acc[v]);
        }
    }
}

// FP: the products of two variable residues in fp64 (f_mulmod with the
// quotient factor w/q formed as w * (1/q): two roundings instead of one, so
// each product lies within 0.875 q of zero for q < 2^50, and eight of them
// sum exactly before a reduction).  Otherwise Barrett products on u64.
// Blocks are numbered so that the ciphertext groups vary fastest: the groups
// that read the same key words run back to back and find them in the cache.
// RAW (fp64 only): the raised limbs in mu are reduced fp64 patterns; the
// digits' own limbs read from x are canonical words either way.
template <bool FP, bool RAW = false>
__device__ __forceinline__ void b_ks_inner(const VBlk &VB, const u64 *__restrict__ mu, const u64 *__restrict__ x, size_t x_ct_stride,
                           const u64 *__restrict__ key, u64 *__restrict__ acc, int level, int nQ, int nmod, int next,
                           int nact, int dnum, int alpha, int count, const PrimeInfo *__restrict__ pinfo, int N) {
    const unsigned lin = VB.x + VB.gx * (VB.y + VB.gy * VB.z);
    const unsigned zg = lin % VB.gz, rest = lin / VB.gz;
    const int n = (int)(rest % VB.gx) * kT + threadIdx.x, e = (int)(rest / VB.gx), ct0 = (int)zg * kKsCts;
    const int prime = ext_prime(e, level, nQ);
    const int own = e <= level ? e / alpha : -1;
    using S = typename std::conditional<FP, double, u64>::type;
    S s0[kKsCts], s1[kKsCts];
#pragma unroll
    for (int c = 0; c < kKsCts; c++) s0[c] = s1[c] = 0;
    const Barrett br = pinfo[prime].br;
    const double q = pinfo[prime].qd, qinv = pinfo[prime].qinv;
    for (int j = 0; j < nact; j++) {
        const u64 *K = key + ((size_t)j * 2 * nmod + prime) * N + n;
        const u64 k0 = K[0], k1 = K[(size_t)nmod * N];
        u64 u[kKsCts];
#pragma unroll
        for (int c = 0; c < kKsCts; c++) {
            const int ct = min(ct0 + c, count - 1);  // a tail thread repeats the last ciphertext
            u[c] = j == own ? x[(size_t)ct * x_ct_stride + (size_t)e * N + n]
                            : mu[(((size_t)ct * dnum + j) * next + e) * N + n];
        }
        if constexpr (FP) {
#pragma clang fp contract(off)
            const double w0 = f_load(k0), w1 = f_load(k1);
            const FPair c0{w0, w0 * qinv}, c1{w1, w1 * qinv};
#pragma unroll
            for (int c = 0; c < kKsCts; c++) {
                const double y = RAW && j != own ? f_raw_load(u[c]) : f_load(u[c]);
                s0[c] += f_mulmod(y, c0, q);
                s1[c] += f_mulmod(y, c1, q);
                if ((j & 7) == 7) {
                    s0[c] = f_reduce(s0[c], q, qinv);
                    s1[c] = f_reduce(s1[c], q, qinv);
                }
            }
        } else {
#pragma unroll
            for (int c = 0; c < kKsCts; c++) {
                s0[c] = add_mod(s0[c], mul_mod(u[c], k0, br), br.q);
                s1[c] = add_mod(s1[c], mul_mod(u[c], k1, br), br.q);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < kKsCts; c++) {
        const int ct = ct0 + c;
        if (ct < count) {
            u64 r0, r1;
            if constexpr (FP) {
                r0 = f_bits(f_canon(s0[c], q, qinv));
                r1 = f_bits(f_canon(s1[c], q, qinv));
            } else {
                r0 = s0[c];
                r1 = s1[c];
            }
            acc[(((size_t)ct * 2 + 0) * next + e) * N + n] = r0;
            acc[(((size_t)ct * 2 + 1) * next + e) * N + n] = r1;
        }
    }
}

// Exact division by P, conversion part (z-grid = ct * 2 + c):
// v_j = [acc_{p_j} p^-1 Phat_j^-1]_{p_j};  TH_i = sum_j v_j Phat_j mod q_i
// (SC: TH_i p P^-1, the constants Phat_j p P^-1 folded, for a consumer that
// subtracts it unscaled).
// With PL > 0 a thread takes the 2^PL words n + v N/2^PL of each limb: it
// applies the last PL stages of the part-limb inverse transform of the
// special limbs to its inputs and the first PL forward stages of TH's
// transforms to its outputs.  FP: fp64 products with the plan's (w, w/q)
// pairs; each product lies within 0.75 q_i of zero (v_j < 2^50), so eight sum
// exactly before a reduction.
template <bool FP, int PL = 0, bool SC = false>
__device__ __forceinline__ void b_moddown(const VBlk &VB, const u64 *__restrict__ acc, u64 *__restrict__ th,
                                          const ModDownPlan *__restrict__ pl, const PrimeInfo *__restrict__ pinfo,
                                          int level, int nQ, int nP, int next, int N) {
    constexpr int NV = 1 << PL, MD = PL > 0 ? kFoldDigit : kMaxDigit;
    const int n = VB.x * kT + threadIdx.x, cc = VB.z, Q = N >> PL;
    const int nl = level + 1;
    const u64 *A = acc + (size_t)cc * next * N + n;
    u64 *T = th + (size_t)cc * nl * N + n;
    if constexpr (!FP) {
        u64 v[NV][MD];
#pragma unroll
        for (int j = 0; j < MD; j++) {
            if (j >= nP) break;
            u64 x[NV];
#pragma unroll
            for (int w = 0; w < NV; w++) x[w] = A[(size_t)(nl + j) * N + w * Q];
            if constexpr (PL > 0) unfold_int<PL>(x, pinfo[nQ + j]);
#pragma unroll
            for (int w = 0; w < NV; w++) v[w][j] = shoup(x[w], pl->vfac[j][0], pl->vfac[j][1], pinfo[nQ + j].q);
        }
        for (int i = 0; i < nl; i++) {
            const PrimeInfo &pi = pinfo[i];
            u64 t[NV];
#pragma unroll
            for (int w = 0; w < NV; w++) {
                t[w] = 0;
#pragma unroll
                for (int j = 0; j < MD; j++) {
                    if (j >= nP) break;
                    const u64 *w2 = SC ? pl->phatpp[i][j] : pl->phat[i][j];
                    t[w] = add_mod(t[w], shoup(v[w][j], w2[0], w2[1], pi.q), pi.q);
                }
            }
            if constexpr (PL > 0) fold_int<PL>(t, pi);
#pragma unroll
            for (int w = 0; w < NV; w++) T[(size_t)i * N + w * Q] = t[w];
        }
    } else {
#pragma clang fp contract(off)
        double v[NV][MD];  // canonical in [0, p_j)
#pragma unroll
        for (int j = 0; j < MD; j++) {
            if (j >= nP) break;
            const PrimeInfo &pj = pinfo[nQ + j];
            double x[NV];
#pragma unroll
            for (int w = 0; w < NV; w++) x[w] = f_load(A[(size_t)(nl + j) * N + w * Q]);
            if constexpr (PL > 0) unfold_fp<PL, false>(x, pj);  // |x| < 1.5 q: fine for the product
#pragma unroll
            for (int w = 0; w < NV; w++) v[w][j] = f_canon(f_mulmod(x[w], fpair(pl->vfac[j]), pj.qd), pj.qd, pj.qinv);
        }
        for (int i = 0; i < nl; i++) {
            const PrimeInfo &pi = pinfo[i];
            double t[NV];
#pragma unroll
            for (int w = 0; w < NV; w++) {
                t[w] = 0.0;
#pragma unroll
                for (int j = 0; j < MD; j++) {
                    if (j >= nP) break;
                    t[w] += f_mulmod(v[w][j], fpair(SC ? pl->phatpp[i][j] : pl->phat[i][j]), pi.qd);
                    if ((j & 7) == 7) t[w] = f_reduce(t[w], pi.qd, pi.qinv);
                }
                // the fold takes |x| < 1.6 q and returns canonical words
                t[w] = PL > 0 ? f_reduce(t[w], pi.qd, pi.qinv) : f_canon(t[w], pi.qd, pi.qinv);
            }
            if constexpr (PL > 0) fold_fp<PL>(t, pi);
#pragma unroll
            for (int w = 0; w < NV; w++) T[(size_t)i * N + w * Q] = f_bits(t[w]);
        }
    }
}

// out_c = base_c + ACC_c P^-1 - TH_c (p P^-1)   (NTT domain, limbs i <= level)
__device__ __forceinline__ void b_ks_combine(const VBlk &VB, const u64 *__restrict__ base0, const u64 *__restrict__ base1, size_t base_ct_stride,
                             const u64 *__restrict__ acc, const u64 *__restrict__ th, u64 *__restrict__ out,
                             size_t out_ct_stride, const ModDownPlan *__restrict__ pl,
                             const PrimeInfo *__restrict__ pinfo, int nl, int next, int N) {
    const int n = VB.x * kT + threadIdx.x, i = VB.y, ct = VB.z;
    const u64 q = pinfo[i].q;
    for (int c = 0; c < 2; c++) {
        u64 a = acc[(((size_t)ct * 2 + c) * next + i) * N + n];
        u64 t = th[(((size_t)ct * 2 + c) * nl + i) * N + n];
        u64 r = sub_mod(shoup(a, pl->pinv[i][0], pl->pinv[i][1], q), shoup(t, pl->ppinv[i][0], pl->ppinv[i][1], q), q);
        const u64 *bp = c == 0 ? base0 : base1;
        if (bp) r = add_mod(r, bp[(size_t)ct * base_ct_stride + (size_t)i * N + n], q);
        out[(size_t)ct * out_ct_stride + ((size_t)c * nl + i) * N + n] = r;
    }
}

// ---------------------- relinearisation fused with one modulus switch
// Coefficient domain, per coefficient and component c (z-grid = ct * 2 + c):
//   th_i  = sum_j v_j Phat_j mod q_i, v_j = [acc_{p_j} p^-1 Phat_j^-1]_{p_j}
//   r_l   = d_l + (acc_l - p th_l) P^-1            (relinearised top limb)
//   t     = [r_l p^-1]_{q_l} in (-q_l/2, q_l/2]
//   E_i   = (th_i p P^-1 + p t) q_l^-1,  i < l
// so that, after E is transformed, out_i = (d_i + acc_i P^-1) q_l^-1 - E_i
// equals the modulus switch of the relinearised ciphertext exactly (every
// step is linear over Z_{q_i}).  d and acc limbs l are coefficient domain here.
// RAW (fp64 only): the accumulator's special and top limbs and d's top limb
// are read, and E is written, as reduced fp64 patterns.
template <bool FP, int PL = 0, int MD = kMaxDigit, bool RAW = false>
__device__ __forceinline__ void b_relin_ms_fbc(const VBlk &VB, const u64 *__restrict__ acc, const u64 *__restrict__ d, size_t d_ct_stride,
                               u64 *__restrict__ E, const ModDownPlan *__restrict__ md,
                               const ModSwitchPlan *__restrict__ ms, const PrimeInfo *__restrict__ pinfo, int level,
                               int nQ, int nP, int next, int N) {
    constexpr int NV = 1 << PL;  // words n + v N/2^PL per thread (PL inverse stages unfolded, PL forward folded)
    const int n = VB.x * kT + threadIdx.x, cc = VB.z, Q = N >> PL;
    const int ct = cc >> 1, c = cc & 1, nl = level + 1;
    const u64 *A = acc + (size_t)cc * next * N + n;
    const u64 *D = d + (size_t)ct * d_ct_stride + ((size_t)c * nl + level) * N + n;
    u64 *Eo = E + (size_t)cc * level * N + n;
    if constexpr (!FP) {
        u64 v[NV][MD], mag[NV];
        bool neg[NV];
        const u64 ql = pinfo[level].q;
        // inputs: the special limbs and the top limb of the accumulator, the
        // top limb of d (the last PL inverse stages applied here when PL > 0)
        u64 sp[NV][MD], top[NV], dt[NV];
#pragma unroll
        for (int j = 0; j < MD; j++) {
            if (j >= nP) break;
            u64 x[NV];
#pragma unroll
            for (int w = 0; w < NV; w++) x[w] = A[(size_t)(nl + j) * N + w * Q];
            if constexpr (PL > 0) unfold_int<PL>(x, pinfo[nQ + j]);
#pragma unroll
            for (int w = 0; w < NV; w++) sp[w][j] = x[w];
        }
#pragma unroll
        for (int w = 0; w < NV; w++) {
            top[w] = A[(size_t)level * N + w * Q];
            dt[w] = D[w * Q];
        }
        if constexpr (PL > 0) {
            unfold_int<PL>(top, pinfo[level]);
            unfold_int<PL>(dt, pinfo[level]);
        }
#pragma unroll
        for (int w = 0; w < NV; w++) {
#pragma unroll
            for (int j = 0; j < MD; j++) {
                if (j >= nP) break;
                v[w][j] = shoup(sp[w][j], md->vfac[j][0], md->vfac[j][1], pinfo[nQ + j].q);
            }
            // top limb of the relinearised component
            u64 th = 0;
#pragma unroll
            for (int j = 0; j < MD; j++) {
                if (j >= nP) break;
                th = add_mod(th, shoup(v[w][j], md->phat[level][j][0], md->phat[level][j][1], ql), ql);
            }
            u64 r = sub_mod(shoup(top[w], md->pinv[level][0], md->pinv[level][1], ql),
                            shoup(th, md->ppinv[level][0], md->ppinv[level][1], ql), ql);
            r = add_mod(r, dt[w], ql);
            const u64 t = shoup(r, ms->pinv_l[0], ms->pinv_l[1], ql);
            neg[w] = t > (ql - 1) / 2;
            mag[w] = neg[w] ? ql - t : t;
        }
        for (int i = 0; i < level; i++) {
            const PrimeInfo &pi = pinfo[i];
            const u64 q = pi.q;
            u64 e[NV];
#pragma unroll
            for (int w = 0; w < NV; w++) {
                u64 h = 0;
#pragma unroll
                for (int j = 0; j < MD; j++) {
                    if (j >= nP) break;
                    h = add_mod(h, shoup(v[w][j], md->phat[i][j][0], md->phat[i][j][1], q), q);
                }
                u64 pt = shoup(mag[w], pi.p_mod, pi.p_modp, q);
                pt = (neg[w] && pt) ? q - pt : pt;
                const u64 x = add_mod(shoup(h, md->ppinv[i][0], md->ppinv[i][1], q), pt, q);
                e[w] = shoup(x, ms->qlinv[i][0], ms->qlinv[i][1], q);
            }
            if constexpr (PL > 0) fold_int<PL>(e, pi);
#pragma unroll
            for (int w = 0; w < NV; w++) Eo[(size_t)i * N + w * Q] = e[w];
        }
    } else {
#pragma clang fp contract(off)
        double v[NV][MD];  // canonical in [0, p_j)
        double t[NV];
        const PrimeInfo &pl = pinfo[level];
        const double ql = pl.qd;
        // inputs: the special limbs and the top limb of the accumulator, the
        // top limb of d (the last PL inverse stages applied here when PL > 0)
        double top[NV], dt[NV];
#pragma unroll
        for (int j = 0; j < MD; j++) {
            if (j >= nP) break;
            const PrimeInfo &pj = pinfo[nQ + j];
            double x[NV];
#pragma unroll
            for (int w = 0; w < NV; w++)
                x[w] = RAW ? f_raw_load(A[(size_t)(nl + j) * N + w * Q]) : f_load(A[(size_t)(nl + j) * N + w * Q]);
            if constexpr (PL > 0) unfold_fp<PL, false>(x, pj);  // |x| < 1.5 q: fine for the product
#pragma unroll
            for (int w = 0; w < NV; w++) v[w][j] = f_canon(f_mulmod(x[w], fpair(md->vfac[j]), pj.qd), pj.qd, pj.qinv);
        }
#pragma unroll
        for (int w = 0; w < NV; w++) {
            top[w] = RAW ? f_raw_load(A[(size_t)level * N + w * Q]) : f_load(A[(size_t)level * N + w * Q]);
            dt[w] = RAW ? f_raw_load(D[w * Q]) : f_load(D[w * Q]);
        }
        if constexpr (PL > 0) {  // |.| < 1.5 q: they enter r below through a product and a sum
            unfold_fp<PL, false>(top, pl);
            unfold_fp<PL, false>(dt, pl);
        }
#pragma unroll
        for (int w = 0; w < NV; w++) {
            double th = 0.0;
#pragma unroll
            for (int j = 0; j < MD; j++) {
                if (j >= nP) break;
                th += f_mulmod(v[w][j], fpair(md->phat[level][j]), ql);
                if ((j & 7) == 7) th = f_reduce(th, ql, pl.qinv);
            }
            th = f_reduce(th, ql, pl.qinv);
            double r = f_mulmod(top[w], fpair(md->pinv[level]), ql) - f_mulmod(th, fpair(md->ppinv[level]), ql) +
                       dt[w];
            // the exact centred lift: it enters every other modulus as an integer
            t[w] = f_centre(f_mulmod(r, fpair(ms->pinv_l), ql), ql, pl.qinv);
        }
        // E_i = (sum_j v_j Phat_j p P^-1 + p t) q_l^-1 with the constants folded
        for (int i = 0; i < level; i++) {
            const PrimeInfo &pi = pinfo[i];
            const double q = pi.qd;
            double e[NV];
#pragma unroll
            for (int w = 0; w < NV; w++) {
                e[w] = f_mulmod(t[w], fpair(ms->rk2[i]), q);
#pragma unroll
                for (int j = 0; j < MD; j++) {
                    if (j >= nP) break;
                    e[w] += f_mulmod(v[w][j], fpair(ms->rk1[i][j]), q);
                    if ((j & 7) == 6) e[w] = f_reduce(e[w], q, pi.qinv);
                }
                // the fold takes |x| < 1.6 q and returns canonical (reduced) words
                e[w] = PL > 0 || RAW ? f_reduce(e[w], q, pi.qinv) : f_canon(e[w], q, pi.qinv);
            }
            if constexpr (PL > 0) fold_fp<PL, !RAW>(e, pi);
#pragma unroll
            for (int w = 0; w < NV; w++) Eo[(size_t)i * N + w * Q] = RAW ? f_raw_bits(e[w]) : f_bits(e[w]);
        }
    }
}

// R[ct][c][i] = p t mod q_i, t = [top p^-1]_{q_l} lifted to (-q_l/2, q_l/2]
template <bool FP, int PL = 0>
__device__ __forceinline__ void b_ms_fbc(const VBlk &VB, const u64 *__restrict__ top, u64 *__restrict__ R, const ModSwitchPlan *__restrict__ pl,
                         const PrimeInfo *__restrict__ pinfo, int level, int N) {
    constexpr int NV = 1 << PL;  // words n + v N/2^PL per thread (PL inverse stages unfolded, PL forward folded)
    const int n = VB.x * kT + threadIdx.x, cc = VB.z, Q = N >> PL;
    const u64 *T = top + (size_t)cc * N + n;
    u64 *Ro = R + (size_t)cc * level * N + n;
    if constexpr (!FP) {
        const u64 ql = pl->ql;
        u64 mag[NV], x[NV];
        bool neg[NV];
#pragma unroll
        for (int w = 0; w < NV; w++) x[w] = T[w * Q];
        if constexpr (PL > 0) unfold_int<PL>(x, pinfo[level]);
#pragma unroll
        for (int w = 0; w < NV; w++) {
            const u64 t = shoup(x[w], pl->pinv_l[0], pl->pinv_l[1], ql);
            neg[w] = t > (ql - 1) / 2;
            mag[w] = neg[w] ? ql - t : t;  // |t| < q_l < q_i
        }
        for (int i = 0; i < level; i++) {
            const PrimeInfo &pi = pinfo[i];
            u64 r[NV];
#pragma unroll
            for (int w = 0; w < NV; w++) {
                r[w] = shoup(mag[w], pi.p_mod, pi.p_modp, pi.q);
                r[w] = (neg[w] && r[w]) ? pi.q - r[w] : r[w];
            }
            if constexpr (PL > 0) fold_int<PL>(r, pi);
#pragma unroll
            for (int w = 0; w < NV; w++) Ro[(size_t)i * N + w * Q] = r[w];
        }
    } else {
        const PrimeInfo &pq = pinfo[level];
        double t[NV];
#pragma unroll
        for (int w = 0; w < NV; w++) t[w] = f_load(T[w * Q]);
        if constexpr (PL > 0) unfold_fp<PL, false>(t, pq);  // |t| < 1.5 q: fine for the product
#pragma unroll
        for (int w = 0; w < NV; w++) t[w] = f_centre(f_mulmod(t[w], fpair(pl->pinv_l), pq.qd), pq.qd, pq.qinv);
        for (int i = 0; i < level; i++) {
            const PrimeInfo &pi = pinfo[i];
            double r[NV];
#pragma unroll
            for (int w = 0; w < NV; w++) {
                r[w] = f_mulmod(t[w], fpair(pi.p_f), pi.qd);  // |r| < 0.65 q
                if constexpr (PL == 0) r[w] = f_canon(r[w], pi.qd, pi.qinv);
            }
            if constexpr (PL > 0) fold_fp<PL>(r, pi);
#pragma unroll
            for (int w = 0; w < NV; w++) Ro[(size_t)i * N + w * Q] = f_bits(r[w]);
        }
    }
}

// out[ct][c][i] = (in - R) q_l^-1, i < level
__device__ __forceinline__ void b_ms_combine(const VBlk &VB, const u64 *__restrict__ in, const u64 *__restrict__ R, u64 *__restrict__ out,
                             const ModSwitchPlan *__restrict__ pl, const PrimeInfo *__restrict__ pinfo, int level,
                             int N) {
    const int n = VB.x * kT + threadIdx.x, i = VB.y, ct = VB.z;
    const u64 q = pinfo[i].q;
    for (int c = 0; c < 2; c++) {
        u64 x = in[(((size_t)ct * 2 + c) * (level + 1) + i) * N + n];
        u64 r = R[(((size_t)ct * 2 + c) * level + i) * N + n];
        out[(((size_t)ct * 2 + c) * level + i) * N + n] = shoup(sub_mod(x, r, q), pl->qlinv[i][0], pl->qlinv[i][1], q);
    }
}

// Component c of ciphertext ct (blockIdx.z = 2 ct + c): babies are read at
// ciphertext ct; outputs go to ciphertext ct0 + ct of a batch of `count` per
// block.
template <bool FP>
__device__ __forceinline__ void b_lincomb(const VBlk &VB, const BabyArg &ba, const u64 *__restrict__ coef, u64 *__restrict__ out, int nbaby, int nblk,
                          int count, int ct0, int nl, const PrimeInfo *__restrict__ pinfo, int N) {
    const int n = VB.x * kT + threadIdx.x, i = VB.y, ct = VB.z >> 1;
    const PrimeInfo &pi = pinfo[i];
    const u64 q = pi.q;
    const size_t L = (size_t)nl * N;
    {
        const int c = VB.z & 1;
        if constexpr (!FP) {
            u64 v[16];
#pragma unroll
            for (int k = 0; k < 16; k++) {
                if (k < nbaby) {
                    const size_t Lk = (size_t)ba.nlb[k] * N;
                    v[k] = ba.baby[k][(size_t)ct * 2 * Lk + (size_t)c * Lk + (size_t)i * N + n];
                }
            }
            for (int t = 0; t < nblk; t++) {
                u64 acc = 0;
#pragma unroll
                for (int k = 0; k < 16; k++) {
                    if (k < nbaby) {
                        const u64 *w = coef + (((size_t)t * nbaby + k) * nl + i) * 2;
                        acc = add_mod(acc, shoup(v[k], w[0], w[1], q), q);
                    }
                }
                out[((size_t)ba.pos[t] * count + ct0 + ct) * 2 * L + (size_t)c * L + (size_t)i * N + n] = acc;
            }
        } else {
#pragma clang fp contract(off)
            const double *cf = reinterpret_cast<const double *>(coef);
            // fully unrolled with uniform guards (a break on the runtime count
            // would leave the loops rolled and index the register arrays
            // through the index mode)
            double hi[16], lo[16];
#pragma unroll
            for (int k = 0; k < 16; k++) {
                if (k < nbaby) {
                    const size_t Lk = (size_t)ba.nlb[k] * N;
                    const double v = f_load(ba.baby[k][(size_t)ct * 2 * Lk + (size_t)c * Lk + (size_t)i * N + n]);
                    hi[k] = __builtin_floor(v * 0x1p-25);
                    lo[k] = __builtin_fma(-hi[k], 0x1p25, v);
                }
            }
            const FPair p25 = fpair(pi.two25_f);
            for (int t = 0; t < nblk; t++) {
                double sh = 0.0, sl = 0.0;
#pragma unroll
                for (int k = 0; k < 16; k++) {
                    if (k < nbaby) {
                        const double w = cf[t * nbaby + k];
                        sh = __builtin_fma(w, hi[k], sh);
                        sl = __builtin_fma(w, lo[k], sl);
                    }
                }
                out[((size_t)ba.pos[t] * count + ct0 + ct) * 2 * L + (size_t)c * L + (size_t)i * N + n] =
                    f_bits(f_canon(f_mulmod(sh, p25, pi.qd) + sl, pi.qd, pi.qinv));
            }
        }
    }
}

// Wide linear combinations with small integer weights (fp64 arithmetic):
// out[k] = sum_{m < M} W[k][m] in[m] (+ c0[k] on component 0) for k < K.
// in holds M blocks of `count` ciphertexts [count][2][nl][N] back to back
// (block stride count 2 nl N words), out K blocks the same way.  W is
// [KT KB][M] doubles (rows past K zero), |W| <= 2^8; c0 is [KT KB] doubles.
// Each input word v < 2^50 is split v = h 2^25 + l; the sums of W h and of
// W l stay below M 2^8 2^25 <= 2^42 (exact in fp64), and the result is
// (sum W h)(2^25 mod q) + sum W l (+ c0), reduced once.  Grid: x = KT N/256
// with the k-tile fastest (the tiles that read the same input words run back
// to back and find them in the cache), y = limb, z = 2 ct + component.
template <int KB>
__device__ __forceinline__ void b_lincomb_wide(const VBlk &VB, const u64 *__restrict__ in, u64 *__restrict__ out,
                                               const double *__restrict__ W, const double *__restrict__ c0, int M,
                                               int K, int KT, int count, int nl,
                                               const PrimeInfo *__restrict__ pinfo, int N) {
#pragma clang fp contract(off)
    const int kt = VB.x % KT, n = (VB.x / KT) * kT + threadIdx.x, i = VB.y, cc = VB.z;
    const size_t blk = (size_t)count * 2 * nl * N;
    const size_t off = (size_t)cc * nl * N + (size_t)i * N + n;
    double sh[KB], sl[KB];
#pragma unroll
    for (int kk = 0; kk < KB; kk++) sh[kk] = sl[kk] = 0.0;
    const double *w = W + (size_t)kt * KB * M;
    for (int m = 0; m < M; m++) {
        const double v = f_load(in[(size_t)m * blk + off]);
        const double h = __builtin_floor(v * 0x1p-25), l = __builtin_fma(-h, 0x1p25, v);
#pragma unroll
        for (int kk = 0; kk < KB; kk++) {
            const double wk = w[(size_t)kk * M + m];
            sh[kk] = __builtin_fma(wk, h, sh[kk]);
            sl[kk] = __builtin_fma(wk, l, sl[kk]);
        }
    }
    const PrimeInfo &pi = pinfo[i];
    const FPair p25 = fpair(pi.two25_f);
    const bool comp0 = (cc & 1) == 0;
#pragma unroll
    for (int kk = 0; kk < KB; kk++) {
        const int k = kt * KB + kk;
        if (k >= K) break;
        double r = f_mulmod(sh[kk], p25, pi.qd) + sl[kk];
        if (comp0) r += c0[k];
        out[(size_t)k * blk + off] = f_bits(f_canon(r, pi.qd, pi.qinv));
    }
}

// The same wide combination on the matrix cores, exactly: every input word
// v < 2^56 is split into eight 7-bit digits x_a (v = sum_a x_a 2^(7a)), and
// for each digit one int8 x int8 -> int32 matrix product
// S_a[k][pos] = sum_m W8[k][m] x_a[m][pos] runs on v_mfma_i32_32x32x32_i8
// (32 outputs x 32 positions, 32 inputs a step): |S_a| <= M 128 127 < 2^23
// for M <= 256.  The weights are W8 = W except where W = 128 (not an int8):
// there W8 = 0 and the input enters through a correction list (`corr`:
// offsets [K + 1], then input indices), added as 128 x mod q.  Recombination
// in fp64: R_lo = sum_{a<4} S_a 2^(7a), R_hi = sum_{a>=4} S_a 2^(7(a-4)), both
// below 2^45 (exact), out = R_hi (2^28 mod q) + R_lo (+ c0) reduced once.
// Block: 256 threads, a tile of 32 positions (one limb of one ciphertext
// component) and all K outputs, wave w taking outputs 32 w .. 32 w + 31.  The
// tile's digits sit in LDS as bytes [8][32][M + 16] (one 16-byte read per
// lane and step).  The weights come as int8 [KP][M] (KP = 128, rows past K
// zero); the A and B operands of a lane cover the same 16 inputs of a step in
// the same byte order, so the products do not depend on how the hardware
// orders them; which output row each accumulator register holds is read once
// from a product whose rows carry their own index.
constexpr int kWideRow = kWideMfmaM + 16;
typedef int v4i_t __attribute__((ext_vector_type(4)));
typedef int v16i_t __attribute__((ext_vector_type(16)));
__device__ __forceinline__ void b_lincomb_wide_mfma(const VBlk &VB, const u64 *__restrict__ in,
                                                    u64 *__restrict__ out, const int8_t *__restrict__ W8,
                                                    const double *__restrict__ c0, const int *__restrict__ corr,
                                                    int M, int K, int count, int nl,
                                                    const PrimeInfo *__restrict__ pinfo, int N,
                                                    unsigned char *__restrict__ lds) {
#pragma clang fp contract(off)
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int i = VB.y, cc = VB.z;
    const int pos0 = VB.x * 32;  // first position of the tile inside the limb
    const size_t blk = (size_t)count * 2 * nl * N;
    const size_t off0 = (size_t)cc * nl * N + (size_t)i * N + pos0;
    const int steps = (M + 31) / 32;
    // the tile's digits into LDS: thread t takes position t % 32 and input
    // quads q = t / 32, t / 32 + 8, ... (four inputs packed per dword)
    {
        const int pp = t & 31;
        for (int q = t >> 5; q < steps * 8; q += 8) {
            u64 w[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int m = 4 * q + j;
                w[j] = m < M ? in[(size_t)m * blk + off0 + pp] : 0;
            }
#pragma unroll
            for (int a = 0; a < 8; a++) {
                u32 d = 0;
#pragma unroll
                for (int j = 0; j < 4; j++) d |= (u32)((w[j] >> (7 * a)) & 127) << (8 * j);
                *reinterpret_cast<u32 *>(lds + ((size_t)a * 32 + pp) * kWideRow + 4 * q) = d;
            }
        }
    }
    __syncthreads();
    const int row_l = lane & 31, half = lane >> 5;  // A row / B column of this lane, its half of a step
    // which output row (inside the wave's 32) each accumulator register holds
    int rowof[16];
    {
        v4i_t a = {0, 0, 0, 0}, b = {0, 0, 0, 0};
        if (half == 0) {
            a[0] = row_l;  // byte 0: this row's index
            b[0] = 1;
        }
        v16i_t z = {0};
        z = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, z, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 16; r++) rowof[r] = z[r];
    }
    const int k0 = wave * 32;
    double rlo[16], rhi[16];
#pragma unroll
    for (int r = 0; r < 16; r++) rlo[r] = rhi[r] = 0.0;
    if (k0 < K) {
        for (int a = 0; a < 8; a++) {
            v16i_t acc = {0};
            for (int st = 0; st < steps; st++) {
                const v4i_t av = *reinterpret_cast<const v4i_t *>(W8 + (size_t)(k0 + row_l) * kWideMfmaM + st * 32 +
                                                                  half * 16);
                const v4i_t bv = *reinterpret_cast<const v4i_t *>(lds + ((size_t)a * 32 + row_l) * kWideRow +
                                                                  st * 32 + half * 16);
                acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(av, bv, acc, 0, 0, 0);
            }
            const double sc = (double)(1 << (7 * (a & 3)));
#pragma unroll
            for (int r = 0; r < 16; r++) {
                if (a < 4) rlo[r] = __builtin_fma((double)acc[r], sc, rlo[r]);
                else rhi[r] = __builtin_fma((double)acc[r], sc, rhi[r]);
            }
        }
        const PrimeInfo &pi = pinfo[i];
        // 2^28 and 128 (both below q) as (w, w/q) pairs
        const double q = pi.qd, u = pi.qinv;
        const double w28 = f_canon(0x1p28, q, u), w128 = 128.0;
        const FPair f28{w28, w28 * u}, f128{w128, w128 * u};
        const bool comp0 = (cc & 1) == 0;
        const int pos = pos0 + row_l;  // this lane's column
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const int k = k0 + rowof[r];
            if (k >= K) continue;
            double v = f_mulmod(rhi[r], f28, q) + rlo[r];
            for (int e = corr[k]; e < corr[k + 1]; e++) {
                const int m = corr[K + 1 + e];
                v += f_mulmod(f_load(in[(size_t)m * blk + (size_t)cc * nl * N + (size_t)i * N + pos]), f128, q);
            }
            if (comp0) v += c0[k];
            out[(size_t)k * blk + (size_t)cc * nl * N + (size_t)i * N + pos] = f_bits(f_canon(v, q, u));
        }
    }
}

// Modulus raising on the matrix cores (fp64 contexts).  For one digit, the
// output word v of target t at base position n (a word of the first PL
// forward stages, like b_modup's fold) is sum over sources s and input words
// v' of y[s][v'](n) * M[t][v][s][v'] mod p_t, M the base-conversion constant
// Qhat_s mod p_t times the fold matrix of the PL stages.  Exact split-int8
// form: y < 2^50 is taken as its bytes y_a (a < 7) shifted to signed
// y_a - 128; the host folds 2^(8a) into the constant and writes each product
// W = M 2^(8a) mod p_t as seven signed base-256 digits w_b (rows (t, v, b),
// columns K = (s, v', a)); v_mfma_i32_32x32x32_i8 sums the byte products
// exactly in int32 (|sum| < 140 * 2^14), and the lane holding the eight rows b
// of a word recombines them in fp64: lo = sum_{b<4} acc_b 2^(8b) (< 2^47),
// hi = sum_{b>=4} acc_b 2^(8(b-4)) (< 2^39), result lo + hi (2^32 mod p_t) +
// C[t][v], C = 128 sum_K W restoring the byte shift.  A block takes 128 base
// positions: phase one writes their input bytes to LDS (row = position, K
// contiguous, STEPS x 32 bytes), phase two gives each of its two waves 64
// positions (two B operands, two independent product chains) and runs every
// target tile of the digit, the next tile's weights loading under the
// current tile's products; the 32 rows of a tile are four words (t, v) x
// eight b, placed so that a lane's sixteen accumulators hold two whole words
// (the 32x32 output layout: register r of lane half h is row
// 8 (r/4) + 4 h + r%4).
constexpr int kMfmaPos = 128;
constexpr int kMfmaThreads = 128;  // two waves, 64 positions (two column tiles) each
template <int PL, bool RAW, int STEPS>
__device__ __forceinline__ void b_modup_mfma(const VBlk &VB, const u64 *__restrict__ xc, u64 *__restrict__ mu,
                                             const ModUpPlan *__restrict__ plans, const int8_t *__restrict__ w8,
                                             const double *__restrict__ corr, int plan_stride, int plan0,
                                             const PrimeInfo *__restrict__ pinfo, int nl, int next, int dnum,
                                             int nmod, int N, unsigned char *__restrict__ lds) {
#pragma clang fp contract(off)
    constexpr int NV = 1 << PL, TPT = 4 / NV, KPAD = 32 * STEPS, KSTRIDE = KPAD + 16;
    const int Q = N >> PL;
    const int ct = VB.z / dnum, j = VB.z - ct * dnum;
    const ModUpPlan &pl = plans[j];
    if (pl.nsrc == 0) return;
    const int n0 = VB.x * kMfmaPos, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const u64 *in = xc + (size_t)ct * nl * N + n0;
#pragma unroll 1
    for (int u = tid; u < kMfmaPos * pl.nsrc; u += kMfmaThreads) {
        const int nn = u & (kMfmaPos - 1), s = u / kMfmaPos;
        const PrimeInfo &pi = pinfo[pl.src_lo + s];
        double x[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) {
            const u64 w = in[(size_t)(pl.src_lo + s) * N + v * Q + nn];
            x[v] = RAW ? f_raw_load(w) : f_load(w);
        }
        if constexpr (PL > 0) unfold_fp<PL, false>(x, pi);
#pragma unroll
        for (int v = 0; v < NV; v++) {
            const double y = f_canon(f_mulmod(x[v], fpair(pl.qhinv[s]), pi.qd), pi.qd, pi.qinv);
            // y + 2^52 carries y in its mantissa; the mask drops the exponent
            // and flips the top bit of every byte (b -> b - 128 as int8)
            const u64 bytes = (u64)__double_as_longlong(y + 0x1p52) ^ 0xC3B0808080808080ull;
            *reinterpret_cast<u64 *>(lds + (size_t)nn * KSTRIDE + (s * NV + v) * 8) = bytes;
        }
    }
    __syncthreads();
    const int row_l = lane & 31, half = lane >> 5;
    v4i_t b0[STEPS], b1[STEPS];
#pragma unroll
    for (int st = 0; st < STEPS; st++) {
        b0[st] = *reinterpret_cast<const v4i_t *>(lds + (size_t)(wave * 64 + row_l) * KSTRIDE + st * 32 + half * 16);
        b1[st] = *reinterpret_cast<const v4i_t *>(lds + (size_t)(wave * 64 + 32 + row_l) * KSTRIDE + st * 32 + half * 16);
    }
    const int8_t *wp = w8 + (size_t)(plan0 + j) * plan_stride + (size_t)row_l * KPAD + half * 16;
    u64 *out = mu + ((size_t)ct * dnum + j) * next * N + n0 + wave * 64 + row_l;
    const int ntiles = (pl.ntgt + TPT - 1) / TPT;
    v4i_t a_cur[STEPS], a_nxt[STEPS];
#pragma unroll
    for (int st = 0; st < STEPS; st++) a_cur[st] = *reinterpret_cast<const v4i_t *>(wp + st * 32);
#pragma unroll 1
    for (int tile = 0; tile < ntiles; tile++) {
        if (tile + 1 < ntiles) {  // the next tile's weights load under this tile's products
#pragma unroll
            for (int st = 0; st < STEPS; st++)
                a_nxt[st] = *reinterpret_cast<const v4i_t *>(wp + (size_t)(tile + 1) * 32 * KPAD + st * 32);
        }
        v16i_t acc[2] = {{0}, {0}};
#pragma unroll
        for (int st = 0; st < STEPS; st++) {
            acc[0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a_cur[st], b0[st], acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a_cur[st], b1[st], acc[1], 0, 0, 0);
        }
#pragma unroll
        for (int k = 0; k < 2; k++) {
            const int unit = 2 * half + k, t = tile * TPT + unit / NV, v = unit % NV;
            if (t >= pl.ntgt) continue;
            const PrimeInfo &pt = pinfo[pl.tgt_prime[t]];
            const double q = pt.qd, u = pt.qinv, c = corr[((size_t)(plan0 + j) * nmod + t) * 4 + v];
            const FPair c32{0x1p32, 0x1p32 * u};
            u64 *o = out + (size_t)pl.tgt_e[t] * N + v * Q;
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const v16i_t &A = acc[h];
                const double lo = __builtin_fma(
                    (double)A[8 * k + 3], 0x1p24,
                    __builtin_fma((double)A[8 * k + 2], 0x1p16, __builtin_fma((double)A[8 * k + 1], 0x1p8, (double)A[8 * k])));
                const double hi = __builtin_fma((double)A[8 * k + 6], 0x1p16,
                                                __builtin_fma((double)A[8 * k + 5], 0x1p8, (double)A[8 * k + 4]));
                double r = (lo + c) + f_mulmod(hi, c32, q);
                r = RAW ? f_reduce(r, q, u) : f_canon(r, q, u);
                o[32 * h] = RAW ? f_raw_bits(r) : f_bits(r);
            }
        }
#pragma unroll
        for (int st = 0; st < STEPS; st++) a_cur[st] = a_nxt[st];
    }
}

}  // namespace

}  // namespace bc
