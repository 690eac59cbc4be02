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

namespace bc {

namespace {

constexpr int kT = 256;

__device__ __forceinline__ int ext_prime(int e, int level, int nQ) { return e <= level ? e : nQ + (e - level - 1); }

// ------------------------------------------------------------ ring ops

// (a0 b0, a0 b1 + a1 b0, a1 b1), plus (c0, c1) on the first two components
// when an addend c is given (a multiply-accumulate's sum before relinearising).
// The output has nl limbs; each operand is read at its own limb count (na,
// nb, nc >= nl): an operand above the output's level contributes its lowest
// nl limbs (level alignment by dropping primes, without a copy).  When b is
// broadcast (bcount < count, ciphertext ct uses b[ct % bcount]) the grid runs
// the count / bcount products that share a b ciphertext back to back, so
// its limbs come from the cache after the first.
template <bool ADD>
__global__ void k_tensor(const u64 *__restrict__ a, const u64 *__restrict__ b, const u64 *__restrict__ c,
                         u64 *__restrict__ out, int bcount, int nl, int na, int nb, int nc,
                         const PrimeInfo *__restrict__ pinfo, int N) {
    const int rep = gridDim.z / bcount;  // products per b ciphertext
    const int n = blockIdx.x * kT + threadIdx.x, i = blockIdx.y;
    const int ct = (int)(blockIdx.z % rep) * bcount + (int)(blockIdx.z / rep);
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
__global__ void k_addsub(const u64 *__restrict__ a, const u64 *__restrict__ b, u64 *__restrict__ out, int bcount,
                         int nl, int na, int nb, int ncomp, int sub, const PrimeInfo *__restrict__ pinfo, int N) {
    const int n = blockIdx.x * kT + threadIdx.x, i = blockIdx.y, ct = blockIdx.z;
    const size_t L = (size_t)nl * N, La = (size_t)na * N, Lb = (size_t)nb * N;
    const u64 q = pinfo[i].q;
    for (int c = 0; c < ncomp; c++) {
        const size_t off = (size_t)i * N + n;
        u64 x = a[(size_t)ct * ncomp * La + c * La + off], y = b[(size_t)(ct % bcount) * ncomp * Lb + c * Lb + off];
        out[(size_t)ct * ncomp * L + c * L + off] = sub ? sub_mod(x, y, q) : add_mod(x, y, q);
    }
}

struct ScalarArg {
    u64 w[kMaxMod][2];
};

__global__ void k_mul_scalar(const u64 *__restrict__ a, u64 *__restrict__ out, int nl, int ncomp, ScalarArg s,
                             const PrimeInfo *__restrict__ pinfo, int N) {
    const int n = blockIdx.x * kT + threadIdx.x, i = blockIdx.y, ct = blockIdx.z;
    const size_t L = (size_t)nl * N;
    const u64 q = pinfo[i].q;
    for (int c = 0; c < ncomp; c++) {
        size_t off = (size_t)ct * ncomp * L + (size_t)c * L + (size_t)i * N + n;
        out[off] = shoup(a[off], s.w[i][0], s.w[i][1], q);
    }
}

// constant polynomial c: every evaluation of component 0 gains c mod q_i
__global__ void k_add_const(const u64 *__restrict__ a, u64 *__restrict__ out, int nl, int ncomp, ScalarArg s,
                            const PrimeInfo *__restrict__ pinfo, int N) {
    const int n = blockIdx.x * kT + threadIdx.x, i = blockIdx.y, ct = blockIdx.z;
    const size_t L = (size_t)nl * N;
    const u64 q = pinfo[i].q;
    for (int c = 0; c < ncomp; c++) {
        size_t off = (size_t)ct * ncomp * L + (size_t)c * L + (size_t)i * N + n;
        u64 x = a[off];
        out[off] = c == 0 ? add_mod(x, s.w[i][0], q) : x;
    }
}

// out[ct][c][i][r] = in[ct][c][i][perm[r]]
__global__ void k_permute(const u64 *__restrict__ in, u64 *__restrict__ out, const u32 *__restrict__ perm, int nl,
                          int ncomp, int N) {
    const int n = blockIdx.x * kT + threadIdx.x, i = blockIdx.y, ct = blockIdx.z;
    const size_t L = (size_t)nl * N;
    const u32 src = perm[n];
    for (int c = 0; c < ncomp; c++) {
        size_t base = (size_t)ct * ncomp * L + (size_t)c * L + (size_t)i * N;
        out[base + n] = in[base + src];
    }
}

// ------------------------------------------------------- key switching

// Fast base conversion of digit j (z-grid = ct * dnum + j):
// y_i = [x_i Qhat_i^-1]_{q_i}, u_t = sum_i y_i Qhat_i mod q_t.
// With PL > 0 a thread takes the 2^PL words n + v N/2^PL of each limb: it
// applies the last PL stages of the part-limb inverse transform that made xc
// to its inputs (unfold_int / unfold_fp) and the first PL forward stages of
// the new limbs' transforms to its outputs (fold_int / fold_fp).  MD bounds
// the digit size at compile time.
template <bool FP, int PL = 0, int MD = kMaxDigit>
__global__ void k_modup(const u64 *__restrict__ xc, u64 *__restrict__ mu, const ModUpPlan *__restrict__ plans,
                        const PrimeInfo *__restrict__ pinfo, int nl, int next, int dnum, int N) {
    constexpr int NV = 1 << PL;
    const int n = blockIdx.x * kT + threadIdx.x, Q = N >> PL;
    const int ct = blockIdx.z / dnum, j = blockIdx.z - ct * dnum;
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
            for (int v = 0; v < NV; v++) x[v] = f_load(in[(size_t)(pl.src_lo + s) * N + v * Q]);
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
                // the fold takes |x| < 1.6 q and returns canonical words
                acc[v] = PL > 0 ? f_reduce(acc[v], pt.qd, pt.qinv) : f_canon(acc[v], pt.qd, pt.qinv);
            }
            if constexpr (PL > 0) fold_fp<PL>(acc, pt);
#pragma unroll
            for (int v = 0; v < NV; v++) out[(size_t)pl.tgt_e[t] * N + v * Q] = f_bits(acc[v]);
        }
    }
}

// ACC[ct][c][e] = sum_j MU[ct][j][e] * K_j,c[prime(e)]   (NTT domain), where
// digit j's own limbs (e in [j alpha, (j+1) alpha)) are X's limbs themselves.
// A thread takes kKsCts consecutive ciphertexts: each key word is read once
// for all of them, and every load is issued before the arithmetic.
constexpr int kKsCts = 8;
// FP: the products of two variable residues in fp64 (f_mulmod with the
// quotient factor w/q formed as w * (1/q): two roundings instead of one, so
// each product lies within 0.875 q of zero for q < 2^50, and eight of them
// sum exactly before a reduction).  Otherwise Barrett products on u64.
// Blocks are numbered so that the ciphertext groups vary fastest: the groups
// that read the same key words run back to back and find them in the cache.
template <bool FP>
__global__ void k_ks_inner(const u64 *__restrict__ mu, const u64 *__restrict__ x, size_t x_ct_stride,
                           const u64 *__restrict__ key, u64 *__restrict__ acc, int level, int nQ, int nmod, int next,
                           int nact, int dnum, int alpha, int count, const PrimeInfo *__restrict__ pinfo, int N) {
    const unsigned lin = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    const unsigned zg = lin % gridDim.z, rest = lin / gridDim.z;
    const int n = (int)(rest % gridDim.x) * kT + threadIdx.x, e = (int)(rest / gridDim.x), ct0 = (int)zg * kKsCts;
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
                const double y = f_load(u[c]);
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
// v_j = [acc_{p_j} p^-1 Phat_j^-1]_{p_j};  TH_i = sum_j v_j Phat_j mod q_i.
__global__ void k_moddown(const u64 *__restrict__ acc, u64 *__restrict__ th, const ModDownPlan *__restrict__ pl,
                          const PrimeInfo *__restrict__ pinfo, int level, int nQ, int nP, int next, int N) {
    const int n = blockIdx.x * kT + threadIdx.x, cc = blockIdx.z;
    const int nl = level + 1;
    u64 v[kMaxDigit];
#pragma unroll
    for (int j = 0; j < kMaxDigit; j++) {
        if (j >= nP) break;
        u64 x = acc[((size_t)cc * next + nl + j) * N + n];
        v[j] = shoup(x, pl->vfac[j][0], pl->vfac[j][1], pinfo[nQ + j].q);
    }
    for (int i = 0; i < nl; i++) {
        const u64 q = pinfo[i].q;
        u64 t = 0;
#pragma unroll
        for (int j = 0; j < kMaxDigit; j++) {
            if (j >= nP) break;
            t = add_mod(t, shoup(v[j], pl->phat[i][j][0], pl->phat[i][j][1], q), q);
        }
        th[((size_t)cc * nl + i) * N + n] = t;
    }
}

// out_c = base_c + ACC_c P^-1 - TH_c (p P^-1)   (NTT domain, limbs i <= level)
__global__ void k_ks_combine(const u64 *__restrict__ base0, const u64 *__restrict__ base1, size_t base_ct_stride,
                             const u64 *__restrict__ acc, const u64 *__restrict__ th, u64 *__restrict__ out,
                             size_t out_ct_stride, const ModDownPlan *__restrict__ pl,
                             const PrimeInfo *__restrict__ pinfo, int nl, int next, int N) {
    const int n = blockIdx.x * kT + threadIdx.x, i = blockIdx.y, ct = blockIdx.z;
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
template <bool FP, int PL = 0, int MD = kMaxDigit>
__global__ void k_relin_ms_fbc(const u64 *__restrict__ acc, const u64 *__restrict__ d, size_t d_ct_stride,
                               u64 *__restrict__ E, const ModDownPlan *__restrict__ md,
                               const ModSwitchPlan *__restrict__ ms, const PrimeInfo *__restrict__ pinfo, int level,
                               int nQ, int nP, int next, int N) {
    constexpr int NV = 1 << PL;  // words n + v N/2^PL per thread (PL inverse stages unfolded, PL forward folded)
    const int n = blockIdx.x * kT + threadIdx.x, cc = blockIdx.z, Q = N >> PL;
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
            for (int w = 0; w < NV; w++) x[w] = f_load(A[(size_t)(nl + j) * N + w * Q]);
            if constexpr (PL > 0) unfold_fp<PL, false>(x, pj);  // |x| < 1.5 q: fine for the product
#pragma unroll
            for (int w = 0; w < NV; w++) v[w][j] = f_canon(f_mulmod(x[w], fpair(md->vfac[j]), pj.qd), pj.qd, pj.qinv);
        }
#pragma unroll
        for (int w = 0; w < NV; w++) {
            top[w] = f_load(A[(size_t)level * N + w * Q]);
            dt[w] = f_load(D[w * Q]);
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
                // the fold takes |x| < 1.6 q and returns canonical words
                e[w] = PL > 0 ? f_reduce(e[w], q, pi.qinv) : f_canon(e[w], q, pi.qinv);
            }
            if constexpr (PL > 0) fold_fp<PL>(e, pi);
#pragma unroll
            for (int w = 0; w < NV; w++) Eo[(size_t)i * N + w * Q] = f_bits(e[w]);
        }
    }
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

// R[ct][c][i] = p t mod q_i, t = [top p^-1]_{q_l} lifted to (-q_l/2, q_l/2]
template <bool FP, int PL = 0>
__global__ void k_ms_fbc(const u64 *__restrict__ top, u64 *__restrict__ R, const ModSwitchPlan *__restrict__ pl,
                         const PrimeInfo *__restrict__ pinfo, int level, int N) {
    constexpr int NV = 1 << PL;  // words n + v N/2^PL per thread (PL inverse stages unfolded, PL forward folded)
    const int n = blockIdx.x * kT + threadIdx.x, cc = blockIdx.z, Q = N >> PL;
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
__global__ void k_ms_combine(const u64 *__restrict__ in, const u64 *__restrict__ R, u64 *__restrict__ out,
                             const ModSwitchPlan *__restrict__ pl, const PrimeInfo *__restrict__ pinfo, int level,
                             int N) {
    const int n = blockIdx.x * kT + threadIdx.x, i = blockIdx.y, ct = blockIdx.z;
    const u64 q = pinfo[i].q;
    for (int c = 0; c < 2; c++) {
        u64 x = in[(((size_t)ct * 2 + c) * (level + 1) + i) * N + n];
        u64 r = R[(((size_t)ct * 2 + c) * level + i) * N + n];
        out[(((size_t)ct * 2 + c) * level + i) * N + n] = shoup(sub_mod(x, r, q), pl->qlinv[i][0], pl->qlinv[i][1], q);
    }
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
// Component c of ciphertext ct (blockIdx.z = 2 ct + c): babies are read at
// ciphertext ct; outputs go to ciphertext ct0 + ct of a batch of `count` per
// block.
template <bool FP>
__global__ void k_lincomb(BabyArg ba, const u64 *__restrict__ coef, u64 *__restrict__ out, int nbaby, int nblk,
                          int count, int ct0, int nl, const PrimeInfo *__restrict__ pinfo, int N) {
    const int n = blockIdx.x * kT + threadIdx.x, i = blockIdx.y, ct = blockIdx.z >> 1;
    const PrimeInfo &pi = pinfo[i];
    const u64 q = pi.q;
    const size_t L = (size_t)nl * N;
    {
        const int c = blockIdx.z & 1;
        if constexpr (!FP) {
            u64 v[16];
#pragma unroll
            for (int k = 0; k < 16; k++) {
                if (k >= nbaby) break;
                const size_t Lk = (size_t)ba.nlb[k] * N;
                v[k] = ba.baby[k][(size_t)ct * 2 * Lk + (size_t)c * Lk + (size_t)i * N + n];
            }
            for (int t = 0; t < nblk; t++) {
                u64 acc = 0;
#pragma unroll
                for (int k = 0; k < 16; k++) {
                    if (k >= nbaby) break;
                    const u64 *w = coef + (((size_t)t * nbaby + k) * nl + i) * 2;
                    acc = add_mod(acc, shoup(v[k], w[0], w[1], q), q);
                }
                out[((size_t)ba.pos[t] * count + ct0 + ct) * 2 * L + (size_t)c * L + (size_t)i * N + n] = acc;
            }
        } else {
#pragma clang fp contract(off)
            const double *cf = reinterpret_cast<const double *>(coef);
            double hi[16], lo[16];
#pragma unroll
            for (int k = 0; k < 16; k++) {
                if (k >= nbaby) break;
                const size_t Lk = (size_t)ba.nlb[k] * N;
                const double v = f_load(ba.baby[k][(size_t)ct * 2 * Lk + (size_t)c * Lk + (size_t)i * N + n]);
                hi[k] = __builtin_floor(v * 0x1p-25);
                lo[k] = __builtin_fma(-hi[k], 0x1p25, v);
            }
            const FPair p25 = fpair(pi.two25_f);
            for (int t = 0; t < nblk; t++) {
                double sh = 0.0, sl = 0.0;
#pragma unroll
                for (int k = 0; k < 16; k++) {
                    if (k >= nbaby) break;
                    const double w = cf[t * nbaby + k];
                    sh = __builtin_fma(w, hi[k], sh);
                    sl = __builtin_fma(w, lo[k], sl);
                }
                out[((size_t)ba.pos[t] * count + ct0 + ct) * 2 * L + (size_t)c * L + (size_t)i * N + n] =
                    f_bits(f_canon(f_mulmod(sh, p25, pi.qd) + sl, pi.qd, pi.qinv));
            }
        }
    }
}

inline dim3 grid3(int N, int y, int z) { return dim3((unsigned)(N / kT), (unsigned)y, (unsigned)z); }

}  // namespace

// ------------------------------------------------------------ launchers

void launch_tensor(const bc_ctx *c, const u64 *a, const u64 *b, const u64 *addend, u64 *out, int count, int bcount,
                   int nl, int na, int nb, int nc, hipStream_t st) {
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
    k_mul_scalar<<<grid3(c->N, nl, count), kT, 0, st>>>(a, out, nl, ncomp, scalar_arg(c, v, nl), c->pinfo, c->N);
}
void launch_add_const(const bc_ctx *c, const u64 *a, u64 *out, int count, int nl, int ncomp, int64_t v, hipStream_t st) {
    k_add_const<<<grid3(c->N, nl, count), kT, 0, st>>>(a, out, nl, ncomp, scalar_arg(c, v, nl), c->pinfo, c->N);
}
void launch_permute(const bc_ctx *c, const u64 *in, u64 *out, const u32 *perm, int count, int nl, int ncomp,
                    hipStream_t st) {
    k_permute<<<grid3(c->N, nl, count), kT, 0, st>>>(in, out, perm, nl, ncomp, c->N);
}
template <bool FP, int PL, int MD>
static void modup_pl(const bc_ctx *c, const u64 *xc, u64 *mu, int count, int level, int next, hipStream_t st) {
    k_modup<FP, PL, MD><<<grid3(c->N >> PL, 1, count * c->dnum), kT, 0, st>>>(
        xc, mu, (FP ? c->modup_f : c->modup) + (size_t)level * c->dnum, c->pinfo, level + 1, next, c->dnum, c->N);
}
template <bool FP>
static void modup_a(const bc_ctx *c, const u64 *xc, u64 *mu, int count, int level, int next, int pl, hipStream_t st) {
    if (pl == 2) modup_pl<FP, 2, kFoldDigit>(c, xc, mu, count, level, next, st);
    else if (pl == 1) modup_pl<FP, 1, kFoldDigit>(c, xc, mu, count, level, next, st);
    else modup_pl<FP, 0, kMaxDigit>(c, xc, mu, count, level, next, st);
}
void launch_modup(const bc_ctx *c, const u64 *xc, u64 *mu, int count, int level, int next, int pl, hipStream_t st) {
    double limbs = 0;  // each digit's source limbs read, its new limbs written
    for (int j = 0; j < c->dnum; j++) {
        const ModUpPlan &p = c->h_modup[(size_t)level * c->dnum + j];
        if (p.nsrc) limbs += p.nsrc + p.ntgt;
    }
    ProfScope ps(c, kProfModUp, 8.0 * c->N * limbs * count, st);
    if (use_fp64(c)) modup_a<true>(c, xc, mu, count, level, next, pl, st);
    else modup_a<false>(c, xc, mu, count, level, next, pl, st);
}
void launch_ks_inner(const bc_ctx *c, const u64 *mu, const u64 *x, size_t x_ct_stride, const u64 *key, u64 *acc,
                     int count, int level, int next, int nact, hipStream_t st) {
    // raised limbs of every active digit read, two accumulators written, the key read once
    ProfScope ps(c, kProfKsInner, 8.0 * c->N * next * ((double)count * (nact + 2) + 2.0 * nact), st);
    const dim3 g = grid3(c->N, next, (count + kKsCts - 1) / kKsCts);
    if (use_fp64(c))
        k_ks_inner<true><<<g, kT, 0, st>>>(mu, x, x_ct_stride, key, acc, level, c->nQ, c->nmod, next, nact, c->dnum,
                                           c->alpha, count, c->pinfo, c->N);
    else
        k_ks_inner<false><<<g, kT, 0, st>>>(mu, x, x_ct_stride, key, acc, level, c->nQ, c->nmod, next, nact, c->dnum,
                                            c->alpha, count, c->pinfo, c->N);
}
void launch_moddown(const bc_ctx *c, const u64 *acc, u64 *th, int count, int level, int next, hipStream_t st) {
    k_moddown<<<grid3(c->N, 1, count * 2), kT, 0, st>>>(acc, th, c->moddown, c->pinfo, level, c->nQ, c->nP, next, c->N);
}
void launch_ks_combine(const bc_ctx *c, const u64 *base0, const u64 *base1, size_t base_ct_stride, const u64 *acc,
                       const u64 *th, u64 *out, size_t out_ct_stride, int count, int level, int next, hipStream_t st) {
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
                            int level, int next, hipStream_t st) {
    k_relin_ms_fbc<FP, PL, MD><<<grid3(c->N >> PL, 1, count * 2), kT, 0, st>>>(
        acc, d, d_ct_stride, E, FP ? c->moddown_f : c->moddown, (FP ? c->modsw_f : c->modsw) + level, c->pinfo, level,
        c->nQ, c->nP, next, c->N);
}
template <bool FP>
static void relin_ms_fbc_a(const bc_ctx *c, const u64 *acc, const u64 *d, size_t d_ct_stride, u64 *E, int count,
                           int level, int next, int pl, hipStream_t st) {
    if (pl == 2) relin_ms_fbc_pl<FP, 2, kFoldDigit>(c, acc, d, d_ct_stride, E, count, level, next, st);
    else if (pl == 1) relin_ms_fbc_pl<FP, 1, kFoldDigit>(c, acc, d, d_ct_stride, E, count, level, next, st);
    else relin_ms_fbc_pl<FP, 0, kMaxDigit>(c, acc, d, d_ct_stride, E, count, level, next, st);
}
void launch_relin_ms_fbc(const bc_ctx *c, const u64 *acc, const u64 *d, size_t d_ct_stride, u64 *E, int count,
                         int level, int next, int pl, hipStream_t st) {
    // per component: the special and top accumulator limbs and d's top limb read, `level` limbs written
    ProfScope ps(c, kProfRelinMs, 8.0 * c->N * 2.0 * count * (c->nP + 2 + level), st);
    if (use_fp64(c)) relin_ms_fbc_a<true>(c, acc, d, d_ct_stride, E, count, level, next, pl, st);
    else relin_ms_fbc_a<false>(c, acc, d, d_ct_stride, E, count, level, next, pl, st);
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
    ProfScope ps(c, kProfLincomb, 8.0 * c->N * 2.0 * nl * nlaunch * (nbaby + nblk), st);
    if (lincomb_small(c))
        k_lincomb<true><<<grid3(c->N, nl, 2 * nlaunch), kT, 0, st>>>(ba, coef, out, nbaby, nblk, count, ct0, nl,
                                                                    c->pinfo, c->N);
    else
        k_lincomb<false><<<grid3(c->N, nl, 2 * nlaunch), kT, 0, st>>>(ba, coef, out, nbaby, nblk, count, ct0, nl, c->pinfo,
                                                                 c->N);
}
void launch_crt_decode(const bc_ctx *c, const u64 *d, uint32_t *out, int count, int nl, hipStream_t st) {
    k_crt_decode<<<grid3(c->N, 1, count), kT, 0, st>>>(d, out, c->garner, c->pinfo, nl, c->p, c->N);
}

}  // namespace bc
