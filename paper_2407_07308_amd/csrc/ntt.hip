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
// two chunks exchange words through LDS once.  Butterflies are Harvey's lazy
// ones (values in [0, 4q) forward, [0, 2q) inverse) with Shoup products by
// precomputed twiddles.

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

struct Tw {
    const u64 *W, *Wp, *Wi, *Wip;
};

__device__ __forceinline__ Tw tables(const u64 *tw, int prime, int N) {
    const u64 *b = tw + (size_t)prime * 4 * N;
    return {b, b + N, b + 2 * N, b + 3 * N};
}

__device__ __forceinline__ u64 *limb_ptr(const LimbSet &ls, int job, int N, int &prime) {
    int poly = job / ls.nlimb, k = job - poly * ls.nlimb;
    prime = ls.prime[k];
    return ls.base + (size_t)poly * ls.poly_stride + (size_t)ls.off[k] * N;
}

__device__ __forceinline__ void ct_bfly(u64 &X, u64 &Y, u64 w, u64 wp, u64 q, u64 q2) {
    u64 x = X >= q2 ? X - q2 : X;
    u64 t = shoup_lazy(Y, w, wp, q);
    X = x + t;
    Y = x - t + q2;
}

__device__ __forceinline__ void gs_bfly(u64 &X, u64 &Y, u64 w, u64 wp, u64 q, u64 q2) {
    u64 u = X + Y;
    u64 d = X - Y + q2;
    X = u >= q2 ? u - q2 : u;
    Y = shoup_lazy(d, w, wp, q);
}

// Forward chunk: stages on line bits [blo, blo + C) (high to low) of the
// 2^C words v[k] at line positions X0 + (k << blo).  For the stage on bit b
// the twiddle index is tbase(b) + (k >> (C - s)), s = (blo + C - 1) - b, with
// tbase(b) = mb(b) + G * 2^(L-1-b) + (X0 >> (b + 1)).
template <int C>
__device__ __forceinline__ void fwd_chunk(u64 *v, const Tw &t, int L, int blo, int X0, int G, int logM, u64 q) {
    const u64 q2 = 2 * q;
#pragma unroll
    for (int s = 0; s < C; s++) {
        const int b = blo + C - 1 - s;
        const int half = 1 << (C - 1 - s);
        const int tb = (1 << (logM - 1 - b)) + (G << (L - 1 - b)) + (X0 >> (b + 1));
#pragma unroll
        for (int blk = 0; blk < (1 << s); blk++) {
            const u64 w = t.W[tb + blk], wp = t.Wp[tb + blk];
#pragma unroll
            for (int j = 0; j < half; j++) ct_bfly(v[blk * 2 * half + j], v[blk * 2 * half + j + half], w, wp, q, q2);
        }
    }
}

// Inverse chunk: stages on bits blo .. blo + C - 1 (low to high).  With
// `scale`, the last stage (the transform's final one, m = 1) folds in N^-1.
template <int C>
__device__ __forceinline__ void inv_chunk(u64 *v, const Tw &t, int L, int blo, int X0, int G, int logM, u64 q,
                                          bool scale, const PrimeInfo &pi) {
    const u64 q2 = 2 * q;
#pragma unroll
    for (int s = 0; s < C; s++) {
        const int b = blo + s;
        const int half = 1 << s;
        const int tb = (1 << (logM - 1 - b)) + (G << (L - 1 - b)) + (X0 >> (b + 1));
#pragma unroll
        for (int blk = 0; blk < (1 << (C - 1 - s)); blk++) {
            const u64 w = t.Wi[tb + blk], wp = t.Wip[tb + blk];
#pragma unroll
            for (int j = 0; j < half; j++) {
                u64 &X = v[blk * 2 * half + j], &Y = v[blk * 2 * half + j + half];
                if (scale && s == C - 1) {
                    u64 u = X + Y, d = X - Y + q2;
                    u64 a = shoup_lazy(u, pi.ninv, pi.ninvp, q), r = shoup_lazy(d, pi.ninvw1, pi.ninvw1p, q);
                    X = a >= q ? a - q : a;
                    Y = r >= q ? r - q : r;
                } else {
                    gs_bfly(X, Y, w, wp, q, q2);
                }
            }
        }
    }
}

// ---------------------------------------------------------------- pass A
// Columns: line = one column of N1 = 2^L1 words (stride N2 in memory), CW
// columns per workgroup.  Twiddle index of the stage on bit b:
// m = 2^(L1-1-b), group = row >> (b+1)  (so logM = L1, G = 0).
template <int L1, bool INV>
__global__ void __launch_bounds__(kThreads) ntt_cols(LimbSet ls, const u64 *__restrict__ tw,
                                                     const PrimeInfo *__restrict__ pinfo, int logN) {
    constexpr int N1 = 1 << L1;
    constexpr int CW = cols_per_block(L1);
    constexpr int CHI = (L1 + 1) / 2, CLO = L1 - CHI;  // chunk on the high / low row bits
    __shared__ u64 s[N1 * CW];
    const int N = 1 << logN, N2 = N >> L1;
    const int colblocks = N2 / CW;
    const int job = blockIdx.x / colblocks, c0 = (blockIdx.x - job * colblocks) * CW;
    int prime;
    u64 *a = limb_ptr(ls, job, N, prime) + c0;
    const PrimeInfo &pi = pinfo[prime];
    const u64 q = pi.q;
    const Tw t = tables(tw, prime, N);
    const int tid = threadIdx.x;
    u64 v[16];

    // Both chunks touch HBM directly: for a fixed k, consecutive threads take
    // consecutive columns of one row, so every access is coalesced; LDS only
    // carries the exchange between the chunks.
    if (!INV) {
        // high row bits first: words at rows X0 + (k << CLO)
        for (int g = tid; g < (1 << CLO) * CW; g += kThreads) {
            const int col = g % CW, X0 = g / CW;
#pragma unroll
            for (int k = 0; k < (1 << CHI); k++) v[k] = a[(size_t)(X0 + (k << CLO)) * N2 + col];
            fwd_chunk<CHI>(v, t, L1, CLO, X0, 0, L1, q);
#pragma unroll
            for (int k = 0; k < (1 << CHI); k++) s[(X0 + (k << CLO)) * CW + col] = v[k];
        }
        __syncthreads();
        for (int g = tid; g < (1 << CHI) * CW; g += kThreads) {
            const int col = g % CW, X0 = (g / CW) << CLO;
#pragma unroll
            for (int k = 0; k < (1 << CLO); k++) v[k] = s[(X0 + k) * CW + col];
            fwd_chunk<CLO>(v, t, L1, 0, X0, 0, L1, q);
#pragma unroll
            for (int k = 0; k < (1 << CLO); k++) a[(size_t)(X0 + k) * N2 + col] = v[k];
        }
    } else {
        // low row bits first: words at rows X0 + k
        for (int g = tid; g < (1 << CHI) * CW; g += kThreads) {
            const int col = g % CW, X0 = (g / CW) << CLO;
#pragma unroll
            for (int k = 0; k < (1 << CLO); k++) v[k] = a[(size_t)(X0 + k) * N2 + col];
            inv_chunk<CLO>(v, t, L1, 0, X0, 0, L1, q, false, pi);
#pragma unroll
            for (int k = 0; k < (1 << CLO); k++) s[(X0 + k) * CW + col] = v[k];
        }
        __syncthreads();
        for (int g = tid; g < (1 << CLO) * CW; g += kThreads) {
            const int col = g % CW, X0 = g / CW;
#pragma unroll
            for (int k = 0; k < (1 << CHI); k++) v[k] = s[(X0 + (k << CLO)) * CW + col];
            inv_chunk<CHI>(v, t, L1, CLO, X0, 0, L1, q, true, pi);
#pragma unroll
            for (int k = 0; k < (1 << CHI); k++) a[(size_t)(X0 + (k << CLO)) * N2 + col] = v[k];
        }
    }
}

// ---------------------------------------------------------------- pass B
// Rows: line = one row of N2 = 2^L2 contiguous words, R rows per workgroup.
// Twiddle index of the stage on bit b in row u: m = N / 2^(b+1),
// group = u * 2^(L2-1-b) + (x >> (b+1))  (logM = logN, G = u).
// LDS rows are padded by one word per 16 so both chunks' accesses avoid
// bank conflicts.
__device__ __forceinline__ int padx(int x) { return x + (x >> 4); }

template <int L2, bool INV>
__global__ void __launch_bounds__(kThreads) ntt_rows(LimbSet ls, const u64 *__restrict__ tw,
                                                     const PrimeInfo *__restrict__ pinfo, int logN) {
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
    const PrimeInfo &pi = pinfo[prime];
    const u64 q = pi.q;
    const Tw t = tables(tw, prime, N);
    const int tid = threadIdx.x;
    u64 v[16];

    if (!INV) {
        for (int g = tid; g < R << CLO; g += kThreads) {
            const int rr = g >> CLO, X0 = g & ((1 << CLO) - 1);
            const u64 *row = a + (size_t)rr * N2;
#pragma unroll
            for (int k = 0; k < (1 << CHI); k++) v[k] = row[X0 + (k << CLO)];
            fwd_chunk<CHI>(v, t, L2, CLO, X0, u0 + rr, logN, q);
#pragma unroll
            for (int k = 0; k < (1 << CHI); k++) s[rr * RS + padx(X0 + (k << CLO))] = v[k];
        }
        __syncthreads();
        const u64 q2 = 2 * q;
        for (int g = tid; g < R << CHI; g += kThreads) {
            const int rr = g >> CHI, X0 = (g & ((1 << CHI) - 1)) << CLO;
#pragma unroll
            for (int k = 0; k < (1 << CLO); k++) v[k] = s[rr * RS + padx(X0 + k)];
            fwd_chunk<CLO>(v, t, L2, 0, X0, u0 + rr, logN, q);
#pragma unroll
            for (int k = 0; k < (1 << CLO); k++) {
                u64 x = v[k];
                x = x >= q2 ? x - q2 : x;
                s[rr * RS + padx(X0 + k)] = x >= q ? x - q : x;
            }
        }
        __syncthreads();
        for (int idx = tid; idx < R * N2; idx += kThreads) {
            int rr = idx >> L2, x = idx & (N2 - 1);
            a[idx] = s[rr * RS + padx(x)];
        }
    } else {
        for (int idx = tid; idx < R * N2; idx += kThreads) {
            int rr = idx >> L2, x = idx & (N2 - 1);
            s[rr * RS + padx(x)] = a[idx];
        }
        __syncthreads();
        for (int g = tid; g < R << CHI; g += kThreads) {
            const int rr = g >> CHI, X0 = (g & ((1 << CHI) - 1)) << CLO;
#pragma unroll
            for (int k = 0; k < (1 << CLO); k++) v[k] = s[rr * RS + padx(X0 + k)];
            inv_chunk<CLO>(v, t, L2, 0, X0, u0 + rr, logN, q, false, pi);
#pragma unroll
            for (int k = 0; k < (1 << CLO); k++) s[rr * RS + padx(X0 + k)] = v[k];
        }
        __syncthreads();
        for (int g = tid; g < R << CLO; g += kThreads) {
            const int rr = g >> CLO, X0 = g & ((1 << CLO) - 1);
#pragma unroll
            for (int k = 0; k < (1 << CHI); k++) v[k] = s[rr * RS + padx(X0 + (k << CLO))];
            inv_chunk<CHI>(v, t, L2, CLO, X0, u0 + rr, logN, q, false, pi);
            u64 *row = a + (size_t)rr * N2;
#pragma unroll
            for (int k = 0; k < (1 << CHI); k++) row[X0 + (k << CLO)] = v[k];
        }
    }
}

template <bool INV>
void launch_cols(int logN1, int logN, const LimbSet &ls, const bc_ctx *c, hipStream_t st) {
    int N2 = 1 << (logN - logN1), C = cols_per_block(logN1);
    int njobs = ls.npoly * ls.nlimb;
    dim3 grid((unsigned)(njobs * (N2 / C)));
#define BC_COLS(L)                                                                                \
    case L:                                                                                       \
        ntt_cols<L, INV><<<grid, kThreads, 0, st>>>(ls, c->tw, c->pinfo, logN);                   \
        break;
    switch (logN1) {
        BC_COLS(5) BC_COLS(6) BC_COLS(7) BC_COLS(8)
        default: throw Error(BC_ERR_PARAM, "ntt: unsupported column length");
    }
#undef BC_COLS
}

template <bool INV>
void launch_rows(int logN2, int logN, const LimbSet &ls, const bc_ctx *c, hipStream_t st) {
    int N1 = 1 << (logN - logN2), R = std::min(kLineWords >> logN2, N1);
    int njobs = ls.npoly * ls.nlimb;
    dim3 grid((unsigned)(njobs * (N1 / R)));
#define BC_ROWS(L)                                                                                \
    case L:                                                                                       \
        ntt_rows<L, INV><<<grid, kThreads, 0, st>>>(ls, c->tw, c->pinfo, logN);                   \
        break;
    switch (logN2) {
        BC_ROWS(5) BC_ROWS(6) BC_ROWS(7) BC_ROWS(8)
        default: throw Error(BC_ERR_PARAM, "ntt: unsupported row length");
    }
#undef BC_ROWS
}

}  // namespace

// Algorithmic bytes of a transform: every limb read once and written once.
static double ntt_bytes(const bc_ctx *c, const LimbSet &ls) { return 16.0 * c->N * ls.npoly * ls.nlimb; }

// N1 = 2^floor(logN/2) rows, N2 = 2^ceil(logN/2) columns.
void ntt_forward(const bc_ctx *c, const LimbSet &ls, hipStream_t st) {
    if (ls.npoly == 0 || ls.nlimb == 0) return;
    int logN1 = c->logN / 2, logN2 = c->logN - logN1;
    ProfRec r{};
    const bool prof = c->prof->on;
    if (prof) c->prof->begin(kProfNttFwd, ntt_bytes(c, ls), st, r);
    launch_cols<false>(logN1, c->logN, ls, c, st);
    launch_rows<false>(logN2, c->logN, ls, c, st);
    if (prof) c->prof->end(r, st);
    BC_HIP(hipGetLastError());
}

void ntt_inverse(const bc_ctx *c, const LimbSet &ls, hipStream_t st) {
    if (ls.npoly == 0 || ls.nlimb == 0) return;
    int logN1 = c->logN / 2, logN2 = c->logN - logN1;
    ProfRec r{};
    const bool prof = c->prof->on;
    if (prof) c->prof->begin(kProfNttInv, ntt_bytes(c, ls), st, r);
    launch_rows<true>(logN2, c->logN, ls, c, st);
    launch_cols<true>(logN1, c->logN, ls, c, st);
    if (prof) c->prof->end(r, st);
    BC_HIP(hipGetLastError());
}

}  // namespace bc
