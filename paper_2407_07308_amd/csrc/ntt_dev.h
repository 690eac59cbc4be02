// ntt_dev.h -- device code of the batched negacyclic NTT / inverse NTT for
// gfx950: arithmetic policies, register chunks, LDS exchanges, and the
// single-pass / part-limb transform body shared by the transform kernels and
// the persistent executor.
//
// Forward: natural-order coefficients in, bit-reversed evaluations out,
// position r holding a(psi^(2 brv(r) + 1)); the stage with butterfly span h
// (m = N / 2h) multiplies group i by W[m + i] = psi^brv(m + i).  Inverse:
// Gentleman-Sande with Winv[k] = W[k]^-1 in the reverse stage order, scaled
// by N^-1 (paper, Background, "Efficient Polynomial and NTT").
#pragma once

#include <algorithm>

#include "bc_internal.h"

namespace bc {

namespace {

constexpr int kThreads = 256;
constexpr int kLineWords = kThreads * 16;  // words of one workgroup (32 KiB): 16 per thread

// Columns per workgroup of pass A (N2 >= N1 always, so this never exceeds N2).
constexpr int cols_per_block(int L1) {
    return (kLineWords >> L1) < (1 << L1) ? (kLineWords >> L1) : (1 << L1);
}

// ------------------------------------------------------------ arithmetic
// The transforms are written once over an arithmetic policy A:
//   A::V                the register type of a word inside a transform
//   load(u64) / store() canonical word in [0, q) <-> register value
//   raw(V) / unraw(u64) register value <-> its 64-bit pattern, for LDS and
//                       for the intermediate between two passes
//   fw(k) / iw(k)       forward / inverse twiddle of table index k
//   ct, gs              one butterfly; gs_last folds N^-1 into the final one
//
// IntA: Harvey's lazy butterflies on u64 with Shoup products (any q < 2^62):
// values in [0, 4q) forward, [0, 2q) inverse.
//
// FpA (every prime below 2^50): words are integers held in doubles, where
// the products run at the full fp64 rate (f_mulmod and f_reduce, exact).
// Values are reduced (prep) at the start of every register chunk (at most
// five stages) except one loaded from canonical words.  Forward butterflies
// are lazy, X +- y w mod q: a stage adds at most q (1/2 + B 2^-52) to the bound
// B, so five stages from B = q stay below 7.2 q.  Inverse butterflies reduce
// the sum on the chunk's odd stages, keeping values below 4 q and sums and
// differences below 6 q.  Everything stays below 2^53 (= 8 q for q < 2^50):
// no step rounds.
struct IntA {
    using V = u64;
    struct T {
        u64 w, wp;
    };
    // twiddles come from the table (a Shoup companion would need a division)
    static constexpr bool kDerive = false;
    __device__ T derive(T a, T) const { return a; }
    __device__ T square(T a) const { return a; }
    const u64 *W, *Wp, *Wi, *Wip;
    u64 q, q2, ninv, ninvp, ninvw1, ninvw1p;
    __device__ IntA(const void *tw, const PrimeInfo &pi, int prime, int N) {
        const u64 *b = static_cast<const u64 *>(tw) + (size_t)prime * 4 * N;
        W = b;
        Wp = b + N;
        Wi = b + 2 * N;
        Wip = b + 3 * N;
        q = pi.q;
        q2 = 2 * q;
        ninv = pi.ninv;
        ninvp = pi.ninvp;
        ninvw1 = pi.ninvw1;
        ninvw1p = pi.ninvw1p;
    }
    __device__ T fw(int k) const { return {W[k], Wp[k]}; }
    __device__ T iw(int k) const { return {Wi[k], Wip[k]}; }
    __device__ V load(u64 x) const { return x; }
    __device__ u64 store(V x) const {
        x = x >= q2 ? x - q2 : x;
        return x >= q ? x - q : x;
    }
    __device__ static u64 raw(V x) { return x; }
    __device__ static V unraw(u64 x) { return x; }
    __device__ V reduce(V x) const { return x; }  // (no reduced fp64 words on this path)
    __device__ V prep(V x) const { return x; }
    __device__ void ct(V &X, V &Y, T t) const {
        u64 x = X >= q2 ? X - q2 : X;
        u64 p = shoup_lazy(Y, t.w, t.wp, q);
        X = x + p;
        Y = x - p + q2;
    }
    __device__ void gs(V &X, V &Y, T t, bool) const {
        u64 u = X + Y, d = X - Y + q2;
        X = u >= q2 ? u - q2 : u;
        Y = shoup_lazy(d, t.w, t.wp, q);
    }
    __device__ void gs_last(V &X, V &Y) const {
        u64 u = X + Y, d = X - Y + q2;
        X = shoup_lazy(u, ninv, ninvp, q);
        Y = shoup_lazy(d, ninvw1, ninvw1p, q);
    }
    __device__ static T pair(const u64 *p) { return {p[0], p[1]}; }
    // d w0 + a w1 - e and (d - e) w0, canonical words in and out
    __device__ u64 combine(u64 d, u64 a, u64 e, T w0, T w1) const {
        return sub_mod(add_mod(shoup(d, w0.w, w0.wp, q), shoup(a, w1.w, w1.wp, q), q), e, q);
    }
    __device__ u64 switch_(u64 d, u64 e, T w0) const { return shoup(sub_mod(d, e, q), w0.w, w0.wp, q); }
};

struct FpA {
    using V = double;
    struct T {
        double w, wq;
    };
    static constexpr bool kDerive = true;
    const double *W, *Wq, *Wi, *Wiq;
    double q, u, ninv, ninvq, ninvw1, ninvw1q;
    __device__ FpA(const void *tw, const PrimeInfo &pi, int prime, int N) {
        const double *b = static_cast<const double *>(tw) + (size_t)prime * 4 * N;
        W = b;
        Wq = b + N;
        Wi = b + 2 * N;
        Wiq = b + 3 * N;
        q = pi.qd;
        u = pi.qinv;
        ninv = pi.ninv_d;
        ninvq = pi.ninv_q;
        ninvw1 = pi.ninvw1_d;
        ninvw1q = pi.ninvw1_q;
    }
    __device__ T fw(int k) const { return {W[k], Wq[k]}; }
    __device__ T iw(int k) const { return {Wi[k], Wiq[k]}; }
    // Derived twiddles.  derive(a, c) = a.w c.w for a multiplier c held
    // centred in the table (|c.w| <= q/2, c.wq = c.w/q correctly rounded): the
    // quotient estimate errs by at most 1/2 + |a.w| 2^-53, so the product lies
    // below q (1/2 + |a.w| 2^-53) <= q (1/2 + 1/8 |a.w|/q) (q < 2^50), and
    // along any chain from a table word (< q) below 5q/8.  Its quotient factor
    // is w * (1/q) (two roundings): a butterfly's estimate y (w/q) then errs
    // by at most 1/2 + |y| (5/8)(3/2) 2^-52 < 1/2 + |y| 2^-52, inside the
    // bound the table's twiddles (canonical, w/q correctly rounded) give.
    __device__ T derive(T a, T c) const {
#pragma clang fp contract(off)
        const double w = mulmod(a.w, c.w, c.wq);
        return {w, w * u};
    }
    // square(a) = a.w^2 for a derived or table a (|a.w| < q): below
    // q (1/2 + 5/32 + 1/16) < 3q/4; its quotient factor corrected by one
    // Newton step (within 2^-53 (1 + 2^-50) of w/q), so the butterfly bound
    // holds (|y| (3/4) 2^-52) and a chain continued from it stays below 5q/8.
    __device__ T square(T a) const {
#pragma clang fp contract(off)
        const double w = mulmod(a.w, a.w, a.wq), k = w * u;
        return {w, __builtin_fma(__builtin_fma(-k, q, w), u, k)};
    }
    __device__ double mulmod(double y, double w, double wq) const { return f_mulmod(y, FPair{w, wq}, q); }
    __device__ double reduce(double x) const { return f_reduce(x, q, u); }
    __device__ V load(u64 x) const { return f_load(x); }
    __device__ u64 store(V x) const { return f_bits(f_canon(x, q, u)); }
    __device__ static u64 raw(V x) { return (u64)__double_as_longlong(x); }
    __device__ static V unraw(u64 x) { return __longlong_as_double((long long)x); }
    __device__ V prep(V x) const { return reduce(x); }
    __device__ void ct(V &X, V &Y, T t) const {
#pragma clang fp contract(off)
        double x = X, p = mulmod(Y, t.w, t.wq);
        X = x + p;
        Y = x - p;
    }
    __device__ void gs(V &X, V &Y, T t, bool red) const {
#pragma clang fp contract(off)
        double s = X + Y, d = X - Y;
        X = red ? reduce(s) : s;
        Y = mulmod(d, t.w, t.wq);
    }
    __device__ void gs_last(V &X, V &Y) const {
#pragma clang fp contract(off)
        double s = X + Y, d = X - Y;
        X = mulmod(s, ninv, ninvq);
        Y = mulmod(d, ninvw1, ninvw1q);
    }
    __device__ static T pair(const u64 *p) {
        return {__longlong_as_double((long long)p[0]), __longlong_as_double((long long)p[1])};
    }
    __device__ u64 combine(u64 d, u64 a, u64 e, T w0, T w1) const {
#pragma clang fp contract(off)
        double r = mulmod(f_load(d), w0.w, w0.wq) + mulmod(f_load(a), w1.w, w1.wq) - f_load(e);
        return store(r);
    }
    __device__ u64 switch_(u64 d, u64 e, T w0) const {
#pragma clang fp contract(off)
        return store(mulmod(f_load(d) - f_load(e), w0.w, w0.wq));
    }
};

// Jobs are ordered limb-major: consecutive workgroups transform the same limb
// of consecutive ciphertexts, so they share one prime's twiddle table and the
// set of tables live in each XCD's L2 at any time stays small.
__device__ __forceinline__ u64 *limb_ptr(const LimbSet &ls, int job, int N, int &prime) {
    int k = job / ls.npoly, poly = job - k * ls.npoly;
    prime = ls.prime[k];
    return ls.base + (size_t)poly * ls.poly_stride + (size_t)ls.off[k] * N;
}
// where the job's words are read (its output limb when in place)
__device__ __forceinline__ const u64 *limb_src(const LimbSet &ls, int job, int N) {
    int k = job / ls.npoly, poly = job - k * ls.npoly;
    if (!ls.ibase) return ls.base + (size_t)poly * ls.poly_stride + (size_t)ls.off[k] * N;
    return ls.ibase + (size_t)poly * ls.ipoly_stride + (size_t)ls.ioff[k] * N;
}

// Forward chunk: stages on line bits [blo, blo + C) (high to low) of the
// 2^C words v[k] at line positions X0 + (k << blo); `fresh`: the words are
// canonical (just loaded), else they are first brought back into range.  For the stage on bit b
// the twiddle index is tbase(b) + (k >> (C - s)), s = (blo + C - 1) - b, with
// tbase(b) = mb(b) + G * 2^(L-1-b) + (X0 >> (b + 1)).
// With NPRE > 0 the twiddles of the first NPRE stages come from pre (stage s,
// group blk at pre[2^s - 1 + blk]), loaded earlier by fwd_twiddles.
template <int C, class A, int NPRE = 0>
__device__ __forceinline__ void fwd_chunk(typename A::V *v, const A &ar, int L, int blo, int X0, int G, int logM,
                                          bool fresh, const typename A::T *pre = nullptr) {
    if (!fresh) {
#pragma unroll
        for (int k = 0; k < (1 << C); k++) v[k] = ar.prep(v[k]);
    }
#pragma unroll
    for (int s = 0; s < C; s++) {
        const int b = blo + C - 1 - s;
        const int half = 1 << (C - 1 - s);
        const int tb = (1 << (logM - 1 - b)) + (G << (L - 1 - b)) + (X0 >> (b + 1));
#pragma unroll
        for (int blk = 0; blk < (1 << s); blk++) {
            const typename A::T w = s < NPRE ? pre[(1 << s) - 1 + blk] : ar.fw(tb + blk);
#pragma unroll
            for (int j = 0; j < half; j++) ar.ct(v[blk * 2 * half + j], v[blk * 2 * half + j + half], w);
        }
    }
}

// Loads the twiddles of the first NPRE stages of fwd_chunk<C> (same indices)
// into pre, so that a caller can issue them before an LDS exchange, whose
// barriers wait only for LDS traffic, and find them arrived afterwards.
template <int C, int NPRE, class A>
__device__ __forceinline__ void fwd_twiddles(typename A::T *pre, const A &ar, int L, int blo, int X0, int G,
                                             int logM) {
#pragma unroll
    for (int s = 0; s < NPRE; s++) {
        const int b = blo + C - 1 - s;
        const int tb = (1 << (logM - 1 - b)) + (G << (L - 1 - b)) + (X0 >> (b + 1));
#pragma unroll
        for (int blk = 0; blk < (1 << s); blk++) pre[(1 << s) - 1 + blk] = ar.fw(tb + blk);
    }
}

// Inverse chunk: stages on bits blo .. blo + C - 1 (low to high).  With
// `scale`, the last stage (the transform's final one, m = 1) folds in N^-1.
template <int C, class A>
__device__ __forceinline__ void inv_chunk(typename A::V *v, const A &ar, int L, int blo, int X0, int G, int logM,
                                          bool scale, bool fresh) {
    if (!fresh) {
#pragma unroll
        for (int k = 0; k < (1 << C); k++) v[k] = ar.prep(v[k]);
    }
#pragma unroll
    for (int s = 0; s < C; s++) {
        const int b = blo + s;
        const int half = 1 << s;
        const int tb = (1 << (logM - 1 - b)) + (G << (L - 1 - b)) + (X0 >> (b + 1));
#pragma unroll
        for (int blk = 0; blk < (1 << (C - 1 - s)); blk++) {
            if (scale && s == C - 1) {
#pragma unroll
                for (int j = 0; j < half; j++) ar.gs_last(v[blk * 2 * half + j], v[blk * 2 * half + j + half]);
            } else {
                const typename A::T w = ar.iw(tb + blk);
#pragma unroll
                for (int j = 0; j < half; j++) ar.gs(v[blk * 2 * half + j], v[blk * 2 * half + j + half], w, s & 1);
            }
        }
    }
}

// ---------------------------------------------------------------- pass A
// Columns: line = one column of N1 = 2^L1 words (stride N2 in memory), CW
// columns per workgroup.  Twiddle index of the stage on bit b:
// m = 2^(L1-1-b), group = row >> (b+1)  (so logM = L1, G = 0).  Forward:
// canonical words in, raw register values out (read by pass B); inverse: raw
// in, canonical out.
template <int L1, bool INV, class A>
__global__ void __launch_bounds__(kThreads) ntt_cols(LimbSet ls, const void *__restrict__ tw,
                                                     const PrimeInfo *__restrict__ pinfo, int logN) {
    using V = typename A::V;
    constexpr int N1 = 1 << L1;
    constexpr int CW = cols_per_block(L1);
    constexpr int CHI = (L1 + 1) / 2, CLO = L1 - CHI;  // chunk on the high / low row bits
    __shared__ u64 s[N1 * CW];
    const int N = 1 << logN, N2 = N >> L1;
    const int colblocks = N2 / CW;
    const int job = blockIdx.x / colblocks, c0 = (blockIdx.x - job * colblocks) * CW;
    int prime;
    u64 *a = limb_ptr(ls, job, N, prime) + c0;
    const u64 *ain = limb_src(ls, job, N) + c0;  // forward: the transform's input
    const A ar(tw, pinfo[prime], prime, N);
    const int tid = threadIdx.x;
    V v[16];

    // Both chunks touch HBM directly: for a fixed k, consecutive threads take
    // consecutive columns of one row, so every access is coalesced; LDS only
    // carries the exchange between the chunks.
    if (!INV) {
        // high row bits first: words at rows X0 + (k << CLO)
        for (int g = tid; g < (1 << CLO) * CW; g += kThreads) {
            const int col = g % CW, X0 = g / CW;
#pragma unroll
            for (int k = 0; k < (1 << CHI); k++) v[k] = ar.load(ain[(size_t)(X0 + (k << CLO)) * N2 + col]);
            fwd_chunk<CHI>(v, ar, L1, CLO, X0, 0, L1, true);
#pragma unroll
            for (int k = 0; k < (1 << CHI); k++) s[(X0 + (k << CLO)) * CW + col] = A::raw(v[k]);
        }
        __syncthreads();
        for (int g = tid; g < (1 << CHI) * CW; g += kThreads) {
            const int col = g % CW, X0 = (g / CW) << CLO;
#pragma unroll
            for (int k = 0; k < (1 << CLO); k++) v[k] = A::unraw(s[(X0 + k) * CW + col]);
            fwd_chunk<CLO>(v, ar, L1, 0, X0, 0, L1, false);
#pragma unroll
            for (int k = 0; k < (1 << CLO); k++) a[(size_t)(X0 + k) * N2 + col] = A::raw(v[k]);
        }
    } else {
        // low row bits first: words at rows X0 + k
        for (int g = tid; g < (1 << CHI) * CW; g += kThreads) {
            const int col = g % CW, X0 = (g / CW) << CLO;
#pragma unroll
            for (int k = 0; k < (1 << CLO); k++) v[k] = A::unraw(a[(size_t)(X0 + k) * N2 + col]);
            inv_chunk<CLO>(v, ar, L1, 0, X0, 0, L1, false, false);
#pragma unroll
            for (int k = 0; k < (1 << CLO); k++) s[(X0 + k) * CW + col] = A::raw(v[k]);
        }
        __syncthreads();
        for (int g = tid; g < (1 << CLO) * CW; g += kThreads) {
            const int col = g % CW, X0 = g / CW;
#pragma unroll
            for (int k = 0; k < (1 << CHI); k++) v[k] = A::unraw(s[(X0 + (k << CLO)) * CW + col]);
            inv_chunk<CHI>(v, ar, L1, CLO, X0, 0, L1, true, false);
#pragma unroll
            for (int k = 0; k < (1 << CHI); k++) a[(size_t)(X0 + (k << CLO)) * N2 + col] = ar.store(v[k]);
        }
    }
}

// ---------------------------------------------------------------- pass B
// Rows: line = one row of N2 = 2^L2 contiguous words, R rows per workgroup.
// Twiddle index of the stage on bit b in row u: m = N / 2^(b+1),
// group = u * 2^(L2-1-b) + (x >> (b+1))  (logM = logN, G = u).
// LDS rows are padded by one word per 16 so both chunks' accesses avoid
// bank conflicts.  Forward: raw in, canonical out; inverse: canonical in, raw
// out.
__device__ __forceinline__ int padx(int x) { return x + (x >> 4); }

template <int L2, bool INV, class A>
__global__ void __launch_bounds__(kThreads) ntt_rows(LimbSet ls, const void *__restrict__ tw,
                                                     const PrimeInfo *__restrict__ pinfo, int logN) {
    using V = typename A::V;
    constexpr int N2 = 1 << L2;
    constexpr int RS = N2 + N2 / 16;  // padded row stride in LDS
    constexpr int CHI = (L2 + 1) / 2, CLO = L2 - CHI;
    constexpr int RMAX = kLineWords / N2;
    __shared__ u64 s[RMAX * RS];
    const int N = 1 << logN, N1 = N >> L2;
    const int R = min(RMAX, N1);
    const int rowblocks = N1 / R;
    const int job = blockIdx.x / rowblocks, u0 = (blockIdx.x - job * rowblocks) * R;
    int prime;
    u64 *a = limb_ptr(ls, job, N, prime) + (size_t)u0 * N2;
    const u64 *ain = limb_src(ls, job, N) + (size_t)u0 * N2;  // inverse: the transform's input
    const A ar(tw, pinfo[prime], prime, N);
    const int tid = threadIdx.x;
    V v[16];

    if (!INV) {
        for (int g = tid; g < R << CLO; g += kThreads) {
            const int rr = g >> CLO, X0 = g & ((1 << CLO) - 1);
            const u64 *row = a + (size_t)rr * N2;
#pragma unroll
            for (int k = 0; k < (1 << CHI); k++) v[k] = A::unraw(row[X0 + (k << CLO)]);
            fwd_chunk<CHI>(v, ar, L2, CLO, X0, u0 + rr, logN, false);
#pragma unroll
            for (int k = 0; k < (1 << CHI); k++) s[rr * RS + padx(X0 + (k << CLO))] = A::raw(v[k]);
        }
        __syncthreads();
        for (int g = tid; g < R << CHI; g += kThreads) {
            const int rr = g >> CHI, X0 = (g & ((1 << CHI) - 1)) << CLO;
#pragma unroll
            for (int k = 0; k < (1 << CLO); k++) v[k] = A::unraw(s[rr * RS + padx(X0 + k)]);
            fwd_chunk<CLO>(v, ar, L2, 0, X0, u0 + rr, logN, false);
#pragma unroll
            for (int k = 0; k < (1 << CLO); k++) s[rr * RS + padx(X0 + k)] = ar.store(v[k]);
        }
        __syncthreads();
        for (int idx = tid; idx < R * N2; idx += kThreads) {
            int rr = idx >> L2, x = idx & (N2 - 1);
            a[idx] = s[rr * RS + padx(x)];
        }
    } else {
        for (int idx = tid; idx < R * N2; idx += kThreads) {
            int rr = idx >> L2, x = idx & (N2 - 1);
            s[rr * RS + padx(x)] = ain[idx];
        }
        __syncthreads();
        for (int g = tid; g < R << CHI; g += kThreads) {
            const int rr = g >> CHI, X0 = (g & ((1 << CHI) - 1)) << CLO;
#pragma unroll
            for (int k = 0; k < (1 << CLO); k++) v[k] = ar.load(s[rr * RS + padx(X0 + k)]);
            inv_chunk<CLO>(v, ar, L2, 0, X0, u0 + rr, logN, false, true);
#pragma unroll
            for (int k = 0; k < (1 << CLO); k++) s[rr * RS + padx(X0 + k)] = A::raw(v[k]);
        }
        __syncthreads();
        for (int g = tid; g < R << CLO; g += kThreads) {
            const int rr = g >> CLO, X0 = g & ((1 << CLO) - 1);
#pragma unroll
            for (int k = 0; k < (1 << CHI); k++) v[k] = A::unraw(s[rr * RS + padx(X0 + (k << CLO))]);
            inv_chunk<CHI>(v, ar, L2, CLO, X0, u0 + rr, logN, false, false);
            u64 *row = a + (size_t)rr * N2;
#pragma unroll
            for (int k = 0; k < (1 << CHI); k++) row[X0 + (k << CLO)] = A::raw(v[k]);
        }
    }
}

// ------------------------------------------------ derived twiddles
// Bit reversal is additive over disjoint bits, so W[z + c] = W[z] W[c]
// whenever c < 2^k and the low k bits of z are zero; and W[y] = W[2y]^2 for
// y < N/2 (brv(2y) = brv(y) / 2, brv(y) even).  The same holds for the
// inverse table.  In the second and third register chunks of the single-pass
// layouts a thread's twiddles of one stage are W[tb + c], c = 0 .. 2^(4-r)-1
// (r the stage's register bit), with the low 4 - r bits of tb zero, and
// consecutive stages' bases satisfy tb(b) = 2 tb(b + 1).  So one table word
// per stage (forward) or per chunk (inverse) suffices: the rest are products
// with W[2^k]^(+-1), visiting c in Gray-code order so that each twiddle is
// one product away from the one before.  This replaces the chunks' dependent
// table loads with arithmetic.
template <class A>
struct GrayC {
    typename A::T up[4], dn[4];  // multiplier when bit k of c turns on / off
};
__device__ __forceinline__ double uniform_f64(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)b), hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <class A>
__device__ __forceinline__ GrayC<A> gray_constants(const A &ar, bool inv) {
    GrayC<A> g;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const typename A::T f = ar.fw(1 << k), i = ar.iw(1 << k);
        const typename A::T u = inv ? i : f, d = inv ? f : i;
        g.up[k] = {uniform_f64(u.w), uniform_f64(u.wq)};
        g.dn[k] = {uniform_f64(d.w), uniform_f64(d.wq)};
    }
    return g;
}
// first twiddle of the stage on line bit b (its index has the low bits that
// number the thread's groups zero)
__device__ __forceinline__ int stage_base(int L, int b, int X0, int G, int logM) {
    return (1 << (logM - 1 - b)) + (G << (L - 1 - b)) + (X0 >> (b + 1));
}
// Forward stages on register bits NS-1 .. 0 of the 32 words v[k] at line
// positions X0 + (k << blo); base[r] = W[stage_base(blo + r)].
template <int NS, class A>
__device__ __forceinline__ void fwd_chunk_d(typename A::V *v, const A &ar, const typename A::T *base,
                                            const GrayC<A> &gc, bool fresh) {
    static_assert(NS >= 1 && NS <= 5, "a chunk covers at most the 32 registers");
    if (!fresh) {
#pragma unroll
        for (int k = 0; k < 32; k++) v[k] = ar.prep(v[k]);
    }
#pragma unroll
    for (int r = NS - 1; r >= 0; r--) {
        const int half = 1 << r;
        typename A::T w = base[r];
#pragma unroll
        for (int i = 0; i < (32 >> (r + 1)); i++) {
            const int g = i ^ (i >> 1);
            if (i > 0) {
                const int k = __builtin_ctz(i);
                w = ar.derive(w, (g >> k) & 1 ? gc.up[k] : gc.dn[k]);
            }
#pragma unroll
            for (int j = 0; j < half; j++) ar.ct(v[(g << (r + 1)) + j], v[(g << (r + 1)) + j + half], w);
        }
    }
}
template <int NS, class A>
__device__ __forceinline__ void fwd_bases(typename A::T *base, const A &ar, int L, int blo, int X0, int G, int logM) {
#pragma unroll
    for (int r = 0; r < NS; r++) base[r] = ar.fw(stage_base(L, blo + r, X0, G, logM));
}
// Inverse stages on register bits 0 .. NS-1; base = Winv[stage_base(blo)]
// (each later stage's base is the square of the one before).
// SCALE: the last stage is the transform's final one (m = 1), N^-1 folded in.
template <int NS, class A, bool SCALE = false>
__device__ __forceinline__ void inv_chunk_d(typename A::V *v, const A &ar, typename A::T base, const GrayC<A> &gc,
                                            bool fresh) {
    static_assert(NS >= 1 && NS <= 5, "a chunk covers at most the 32 registers");
    if (!fresh) {
#pragma unroll
        for (int k = 0; k < 32; k++) v[k] = ar.prep(v[k]);
    }
#pragma unroll
    for (int r = 0; r < NS; r++) {
        const int half = 1 << r;
        if (SCALE && r == NS - 1) {
#pragma unroll
            for (int j = 0; j < half; j++) ar.gs_last(v[j], v[j + half]);
            break;
        }
        if (r > 0) base = ar.square(base);
        typename A::T w = base;
#pragma unroll
        for (int i = 0; i < (32 >> (r + 1)); i++) {
            const int g = i ^ (i >> 1);
            if (i > 0) {
                const int k = __builtin_ctz(i);
                w = ar.derive(w, (g >> k) & 1 ? gc.up[k] : gc.dn[k]);
            }
#pragma unroll
            for (int j = 0; j < half; j++) ar.gs(v[(g << (r + 1)) + j], v[(g << (r + 1)) + j + half], w, r & 1);
        }
    }
}

// ------------------------------------------------------------ single pass
// One workgroup of N/32 threads transforms a whole limb (N = 2^12 .. 2^15):
// 32 words per thread in registers, three register chunks on the bit ranges
// [LOGN-5, LOGN), [C3, C3+5) and [0, C3) (C3 = LOGN - 10), two LDS exchanges
// between them.  Every word crosses HBM once in and once out.  At N = 2^15
// the 256 KiB limb does not fit in LDS, so each exchange runs in two rounds
// split on bit 14 of the word index (128 KiB each).
struct alignas(16) U64x2 {
    u64 a, b;
};

constexpr int kSplitWords = 16384;

// LDS slot of word x.  With SPLIT the exchange runs in two rounds on bit BIT
// of x (removed from the slot index); BIT is chosen so that in both layouts it
// is a bit of the thread id, i.e. every thread writes and reads in one round.
// One pad word per 32 keeps the strided accesses conflict-free.  For every
// access below, x = base(thread) + (k << S) with the bits of k << S disjoint
// from the base's and aligned so that lds_pos(base + (k << S)) =
// lds_pos(base) + lds_pos(k << S): the slot is a per-thread base plus a
// compile-time offset (an immediate of the LDS instruction).
template <bool SPLIT, int BIT>
__host__ __device__ constexpr int lds_pos(int x) {
    int y = SPLIT ? (((x >> (BIT + 1)) << BIT) | (x & ((1 << BIT) - 1))) : x;
    return y + (y >> 5);
}
template <bool SPLIT, int BIT>
__host__ __device__ constexpr int lds_round(int x) {
    return SPLIT ? (x >> BIT) & 1 : 0;
}

// In the last layout lane l of a wave holds words l*32 .. l*32+31 of the
// wave's 2048-word block, so direct 16-byte accesses would touch 64 cache
// lines per instruction.  These move a wave's block between registers and HBM
// through a wave-private LDS tile (16 x 64 words, rows padded to 65) in two
// halves of 16 registers, every instruction then covering eight whole
// 128-byte lines: in half r, instruction j, lane m handles words 2p, 2p+1
// (p = m % 8) of lane s = 8j + m / 8's sixteen.  Needs 1040 LDS words per
// wave and no workgroup barrier: only the wave touches its tile.
constexpr int kTileRow = 65;

// Epilogue of a forward transform of one E limb (NttCombine): the limb's d,
// acc and out words and its constants.
template <class A>
struct McLimb {
    const u64 *d, *acc;
    u64 *out;
    typename A::T w0, w1;
};

// ROUT: words stored as their reduced fp64 pattern (|x| <= q/2, see ntt_full_body)
// With an epilogue the loads of d and acc for kStoreGroup<EPI> tile rows are
// issued together before their combinations are stored (each word is read and
// then written by the same lane, so an output that is its own d stays
// correct).  The part-limb kernels of the rotation's key switch (a base
// pointer that depends on the component) spilled with groups of four.
template <int EPI>
constexpr int kStoreGroup = EPI == kNttKsCombine ? 2 : 4;
template <class A, int EPI = 0, bool ROUT = false>
__device__ __forceinline__ void store_block(u64 *blk, const typename A::V *v, const A &ar, u64 *tile, int lane,
                                            const McLimb<A> *mc = nullptr, int boff = 0) {
#pragma unroll
    for (int r = 0; r < 2; r++) {
#pragma unroll
        for (int i = 0; i < 16; i++) tile[i * kTileRow + lane] = ROUT ? A::raw(ar.reduce(v[16 * r + i])) : ar.store(v[16 * r + i]);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const int p = lane & 7;
        if constexpr (EPI == 0) {
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const int sl = 8 * j + (lane >> 3), wi = sl * 32 + 16 * r + 2 * p;
                *reinterpret_cast<U64x2 *>(blk + wi) = U64x2{tile[(2 * p) * kTileRow + sl], tile[(2 * p + 1) * kTileRow + sl]};
            }
        } else {
            constexpr int G = kStoreGroup<EPI>;
#pragma unroll
            for (int j0 = 0; j0 < 8; j0 += G) {
                U64x2 dv[G], av[G];
#pragma unroll
                for (int g = 0; g < G; g++) {
                    const int x = boff + (8 * (j0 + g) + (lane >> 3)) * 32 + 16 * r + 2 * p;  // word of the limb
                    dv[g] = *reinterpret_cast<const U64x2 *>(mc->d + x);
                    if constexpr (EPI != kNttSwitch) av[g] = *reinterpret_cast<const U64x2 *>(mc->acc + x);
                }
#pragma unroll
                for (int g = 0; g < G; g++) {
                    const int sl = 8 * (j0 + g) + (lane >> 3), x = boff + sl * 32 + 16 * r + 2 * p;
                    const U64x2 w{tile[(2 * p) * kTileRow + sl], tile[(2 * p + 1) * kTileRow + sl]};
                    U64x2 o;
                    if constexpr (EPI == kNttSwitch) {
                        o = U64x2{ar.switch_(dv[g].a, w.a, mc->w0), ar.switch_(dv[g].b, w.b, mc->w0)};
                    } else {
                        o = U64x2{ar.combine(dv[g].a, av[g].a, w.a, mc->w0, mc->w1),
                                  ar.combine(dv[g].b, av[g].b, w.b, mc->w0, mc->w1)};
                    }
                    *reinterpret_cast<U64x2 *>(mc->out + x) = o;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
}

// Every global load of the block is issued before the first tile pass (the
// second half's loads would otherwise wait behind the first half's LDS work).
template <class A, bool RIN = false>
__device__ __forceinline__ void load_block(const u64 *blk, typename A::V *v, const A &ar, u64 *tile, int lane) {
    const int p = lane & 7;
    U64x2 w[2][8];
#pragma unroll
    for (int r = 0; r < 2; r++) {
#pragma unroll
        for (int j = 0; j < 8; j++) w[r][j] = *reinterpret_cast<const U64x2 *>(blk + (8 * j + (lane >> 3)) * 32 + 16 * r + 2 * p);
    }
#pragma unroll
    for (int r = 0; r < 2; r++) {
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int sl = 8 * j + (lane >> 3);
            tile[(2 * p) * kTileRow + sl] = w[r][j].a;
            tile[(2 * p + 1) * kTileRow + sl] = w[r][j].b;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
        for (int i = 0; i < 16; i++) v[16 * r + i] = RIN ? A::unraw(tile[i * kTileRow + lane]) : ar.load(tile[i * kTileRow + lane]);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
}

// LDS words of ntt_full_body<LOGN, ..., PL> (the exchange buffer; the wave
// tiles of the last layout reuse it).
__host__ __device__ constexpr int ntt_lds_words(int logn, int pl, bool split = false) {
    return (split || pl > 0 || (1 << logn) > kSplitWords ? (1 << logn) / 2 : (1 << logn)) * 33 / 32;
}

// PL > 0: the block transforms one of 2^PL parts of a limb of 2^PL N words.
// Forward: the producer of the words has already applied the first PL
// stages, and what remains are the stages on bits LOGN-1 .. 0, whose
// twiddles are those of the full transform's group `hh` (G = hh, logM =
// LOGN + PL).  Inverse: the stages on bits 0 .. LOGN-1 of the part, without
// N^-1; the consumer of the words applies the last PL stages.  Parts always
// exchange in two rounds, so several blocks share a CU.
// SPL: exchange in two rounds even where the whole buffer would fit (half the
// LDS, for callers that share it with other bodies).
// RIN / ROUT (fp64 arithmetic only): the limbs are read / written as the bit
// patterns of integer-valued doubles instead of canonical words; written ones
// are reduced to |x| <= q/2 (one f_reduce instead of the canonical form and
// its integer conversion).  Such words pass between the key-switching
// kernels only; every consumer takes |x| <= q/2 where it takes [0, q).
template <int LOGN, bool INV, class A, int EPI, int PL = 0, bool SPL = false, bool RIN = false, bool ROUT = false>
__device__ __forceinline__ void ntt_full_body(const LimbSet &ls, const void *__restrict__ tw,
                                              const PrimeInfo *__restrict__ pinfo, const NttCombine *cb, int bid,
                                              u64 *__restrict__ s) {
    using V = typename A::V;
    static_assert(!(RIN || ROUT) || A::kDerive, "reduced fp64 words need the fp64 arithmetic");
    static_assert(!(ROUT && EPI != 0), "an epilogue stores canonical words");
    constexpr int N = 1 << LOGN, C3 = LOGN - 10;
    constexpr bool SP = SPL || PL > 0 || N > kSplitWords;
    constexpr int NSPLIT = SP ? 2 : 1;
    constexpr int NL = N << PL;        // words of the limb
    constexpr int G3 = 1 << (5 - C3);  // chunk-3 groups per thread
    constexpr int LW = SP ? N / 2 : N;
    static_assert(LW + LW / 32 == ntt_lds_words(LOGN, PL, SPL), "LDS size");
    const int t = threadIdx.x;
    const int job = bid >> PL, hh = bid & ((1 << PL) - 1);
    constexpr int LOGM = LOGN + PL;
    int prime;
    u64 *a = limb_ptr(ls, job, NL, prime) + hh * N;
    const u64 *ain = limb_src(ls, job, NL) + hh * N;
    const A ar(tw, pinfo[prime], prime, NL);
    // word index of register k in each layout
    const int x1 = t;                                                     // + (k << (LOGN - 5))
    const int x2 = ((t >> C3) << (C3 + 5)) | (t & ((1 << C3) - 1));       // + (k << C3)
    const int x3 = t << 5;                                                // + k
    V v[32];

    // exchange 1-2 splits on bit C3-1 (a bit of t in both layouts), exchange
    // 2-3 on bit LOGN-1 (t's bit LOGN-6 in both layouts)
    constexpr int BA = C3 - 1, BB = LOGN - 1;
    const int ra = lds_round<SP, BA>(x1), rb = lds_round<SP, BB>(x3);
    const int pa1 = lds_pos<SP, BA>(x1), pa2 = lds_pos<SP, BA>(x2);  // exchange 1-2 bases
    const int pb2 = lds_pos<SP, BB>(x2), pb3 = lds_pos<SP, BB>(x3);  // exchange 2-3 bases
    // chunks 2 and 3 derive their twiddles (fp64 arithmetic); their table
    // words are loaded before the exchange in front of them
    constexpr bool DER = A::kDerive;
    GrayC<A> gc;
    if constexpr (DER) gc = gray_constants(ar, INV);
    if (!INV) {
#pragma unroll
        for (int k = 0; k < 32; k++) v[k] = RIN ? A::unraw(ain[x1 + (k << (LOGN - 5))]) : ar.load(ain[x1 + (k << (LOGN - 5))]);
        // the first chunk's twiddles are the same for every thread: from the
        // table (deriving them was timed slower here, faster in the inverse)
        fwd_chunk<5>(v, ar, LOGN, LOGN - 5, x1, hh, LOGM, true);
        // with an epilogue, the next chunk's first two stages' twiddles travel
        // during the exchange (timed faster there; the plain transform, with
        // fewer registers to spare, was timed slower with it)
        constexpr int NPRE = DER ? 0 : EPI != 0 ? 2 : 0;
        typename A::T pre[3], b2[5];
        if constexpr (NPRE > 0) fwd_twiddles<5, NPRE>(pre, ar, LOGN, C3, x2, hh, LOGM);
        if constexpr (DER) fwd_bases<5>(b2, ar, LOGN, C3, x2, hh, LOGM);
#pragma unroll
        for (int r = 0; r < NSPLIT; r++) {
            if (ra == r) {
#pragma unroll
                for (int k = 0; k < 32; k++) s[pa1 + lds_pos<SP, BA>(k << (LOGN - 5))] = A::raw(v[k]);
            }
            __syncthreads();
            if (ra == r) {
#pragma unroll
                for (int k = 0; k < 32; k++) v[k] = A::unraw(s[pa2 + lds_pos<SP, BA>(k << C3)]);
            }
            __syncthreads();
        }
        if constexpr (DER) fwd_chunk_d<5>(v, ar, b2, gc, false);
        else fwd_chunk<5, A, NPRE>(v, ar, LOGN, C3, x2, hh, LOGM, false, pre);
        typename A::T b3[C3];
        if constexpr (DER) fwd_bases<C3>(b3, ar, LOGN, 0, x3, hh, LOGM);
#pragma unroll
        for (int r = 0; r < NSPLIT; r++) {
            if (rb == r) {
#pragma unroll
                for (int k = 0; k < 32; k++) s[pb2 + lds_pos<SP, BB>(k << C3)] = A::raw(v[k]);
            }
            __syncthreads();
            if (rb == r) {
#pragma unroll
                for (int k = 0; k < 32; k++) v[k] = A::unraw(s[pb3 + lds_pos<SP, BB>(k)]);
            }
            __syncthreads();
        }
        if constexpr (DER) {
            fwd_chunk_d<C3>(v, ar, b3, gc, false);
        } else {
#pragma unroll
            for (int j = 0; j < G3; j++) fwd_chunk<C3>(v + (j << C3), ar, LOGN, 0, x3 + (j << C3), hh, LOGM, false);
        }
        // the exchange above ended with a barrier: LDS is free for the wave tiles
        const int wave = t >> 6, lane = t & 63;
        if constexpr (EPI != 0) {
            const int k = job / ls.npoly, ct = job - k * ls.npoly;
            const int cc = ls.off[k] / cb->level, i = ls.off[k] - cc * cb->level;
            McLimb<A> mc;
            if constexpr (EPI == kNttKsCombine)  // the bases: level limbs per component
                mc.d = cc == 0 ? cb->d + (size_t)ct * cb->d_ct_stride + (size_t)i * NL + hh * N
                               : cb->d1 + (size_t)ct * cb->d1_ct_stride + (size_t)i * cb->d1_limb + hh * N;
            else
                mc.d = cb->d + (size_t)ct * cb->d_ct_stride + ((size_t)cc * (cb->level + 1) + i) * NL + hh * N;
            mc.acc = EPI != kNttSwitch ? cb->acc + (((size_t)ct * 2 + cc) * cb->next + i) * NL + hh * N : nullptr;
            mc.out = cb->out + (((size_t)ct * 2 + cc) * cb->level + i) * NL + hh * N;
            mc.w0 = A::pair(cb->w[i]);
            mc.w1 = A::pair(cb->w[i] + 2);
            store_block<A, EPI>(nullptr, v, ar, s + wave * 16 * kTileRow, lane, &mc, wave << 11);
        } else {
            store_block<A, 0, ROUT>(a + (wave << 11), v, ar, s + wave * 16 * kTileRow, lane);
        }
    } else {
        const int wave = t >> 6, lane = t & 63;
        load_block<A, RIN>(ain + (wave << 11), v, ar, s + wave * 16 * kTileRow, lane);
        __syncthreads();  // every wave is done with its tile before the exchanges reuse LDS
        if constexpr (DER) {
            inv_chunk_d<C3>(v, ar, ar.iw(stage_base(LOGN, 0, x3, hh, LOGM)), gc, true);
        } else {
#pragma unroll
            for (int j = 0; j < G3; j++)
                inv_chunk<C3>(v + (j << C3), ar, LOGN, 0, x3 + (j << C3), hh, LOGM, false, true);
        }
        typename A::T b2{};
        if constexpr (DER) b2 = ar.iw(stage_base(LOGN, C3, x2, hh, LOGM));
#pragma unroll
        for (int r = 0; r < NSPLIT; r++) {
            if (rb == r) {
#pragma unroll
                for (int k = 0; k < 32; k++) s[pb3 + lds_pos<SP, BB>(k)] = A::raw(v[k]);
            }
            __syncthreads();
            if (rb == r) {
#pragma unroll
                for (int k = 0; k < 32; k++) v[k] = A::unraw(s[pb2 + lds_pos<SP, BB>(k << C3)]);
            }
            __syncthreads();
        }
        if constexpr (DER) inv_chunk_d<5>(v, ar, b2, gc, false);
        else inv_chunk<5>(v, ar, LOGN, C3, x2, hh, LOGM, false, false);
        typename A::T b1{};
        if constexpr (DER) b1 = ar.iw(stage_base(LOGN, LOGN - 5, x1, hh, LOGM));
#pragma unroll
        for (int r = 0; r < NSPLIT; r++) {
            if (ra == r) {
#pragma unroll
                for (int k = 0; k < 32; k++) s[pa2 + lds_pos<SP, BA>(k << C3)] = A::raw(v[k]);
            }
            __syncthreads();
            if (ra == r) {
#pragma unroll
                for (int k = 0; k < 32; k++) v[k] = A::unraw(s[pa1 + lds_pos<SP, BA>(k << (LOGN - 5))]);
            }
            __syncthreads();
        }
        if constexpr (DER) inv_chunk_d<5, A, PL == 0>(v, ar, b1, gc, false);
        else inv_chunk<5>(v, ar, LOGN, LOGN - 5, x1, hh, LOGM, PL == 0, false);
#pragma unroll
        for (int k = 0; k < 32; k++) a[x1 + (k << (LOGN - 5))] = ROUT ? A::raw(ar.reduce(v[k])) : ar.store(v[k]);
    }
}

}  // namespace

}  // namespace bc
