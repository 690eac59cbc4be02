// ntt.hip -- batched negacyclic NTT / inverse NTT for gfx950.
//
// The residue polynomials of a ciphertext are multiplied in the evaluation
// domain (paper, Background, "Efficient Polynomial and NTT": radix-2
// Cooley-Tukey forward and Gentleman-Sande inverse transforms for power-of-two
// N).  Forward: natural-order coefficients in, bit-reversed evaluations out,
// position r holding a(psi^(2 brv(r) + 1)); stage m (m = 1, 2, ..., N/2)
// multiplies by W[m + i] = psi^brv(m + i) for butterfly group i.  Inverse:
// Gentleman-Sande with Winv[k] = W[k]^-1, stages m = N/2 .. 1, scaled by N^-1.
//
// A limb of N = N1 * N2 words is treated as an N1 x N2 row-major matrix.  The
// first log2 N1 forward stages only mix words of one column (butterfly span
// >= N2); the remaining log2 N2 stages only mix words of one row.  Pass A
// stages 16 columns of one limb in LDS, pass B stages whole rows; the inverse
// runs B then A.  Each pass reads and writes every word once.  Butterflies are
// Harvey's lazy ones: values live in [0, 4q) (forward) or [0, 2q) (inverse)
// until the last stage, with Shoup multiplications by precomputed twiddles.

#include <algorithm>

#include "bc_internal.h"

namespace bc {

namespace {

constexpr int kThreads = 256;
constexpr int kLdsWords = 2048;  // 16 KiB of LDS per workgroup

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

// ---------------------------------------------------------------- pass A
// One workgroup: C consecutive columns of one limb (N1 words each).
template <int LOGN1, bool INVERSE>
__global__ void __launch_bounds__(kThreads) ntt_pass_cols(LimbSet ls, const u64 *__restrict__ tw,
                                                          const PrimeInfo *__restrict__ pinfo, int logN) {
    constexpr int N1 = 1 << LOGN1;
    constexpr int C = (N1 * 16 <= kLdsWords) ? 16 : kLdsWords / N1;
    __shared__ u64 s[N1 * C];
    const int N = 1 << logN, N2 = N >> LOGN1;
    const int colblocks = N2 / C;
    const int job = blockIdx.x / colblocks, c0 = (blockIdx.x - job * colblocks) * C;
    int prime;
    u64 *a = limb_ptr(ls, job, N, prime);
    const u64 q = pinfo[prime].q, q2 = 2 * q;
    const Tw t = tables(tw, prime, N);
    const int tid = threadIdx.x;

    for (int idx = tid; idx < N1 * C; idx += kThreads) {
        int r = idx / C, c = idx - r * C;
        s[idx] = a[(size_t)r * N2 + c0 + c];
    }
    __syncthreads();

    if (!INVERSE) {
        for (int m = 1, tc = N1 / 2; m < N1; m <<= 1, tc >>= 1) {
            for (int bf = tid; bf < (N1 / 2) * C; bf += kThreads) {
                int c = bf % C, k = bf / C;
                int i = k / tc, j = k - i * tc;
                int r0 = 2 * i * tc + j, r1 = r0 + tc;
                u64 w = t.W[m + i], wp = t.Wp[m + i];
                u64 X = s[r0 * C + c], Y = s[r1 * C + c];
                X = X >= q2 ? X - q2 : X;
                u64 T = shoup_lazy(Y, w, wp, q);
                s[r0 * C + c] = X + T;
                s[r1 * C + c] = X - T + q2;
            }
            __syncthreads();
        }
        for (int idx = tid; idx < N1 * C; idx += kThreads) {
            int r = idx / C, c = idx - r * C;
            a[(size_t)r * N2 + c0 + c] = s[idx];
        }
    } else {
        const PrimeInfo &pi = pinfo[prime];
        for (int m = N1 / 2, tc = 1; m >= 1; m >>= 1, tc <<= 1) {
            for (int bf = tid; bf < (N1 / 2) * C; bf += kThreads) {
                int c = bf % C, k = bf / C;
                int i = k / tc, j = k - i * tc;
                int r0 = 2 * i * tc + j, r1 = r0 + tc;
                u64 X = s[r0 * C + c], Y = s[r1 * C + c];
                u64 U = X + Y;
                U = U >= q2 ? U - q2 : U;
                u64 D = X - Y + q2;
                if (m > 1) {
                    s[r0 * C + c] = U;
                    s[r1 * C + c] = shoup_lazy(D, t.Wi[m + i], t.Wip[m + i], q);
                } else {  // last stage: fold in N^-1 and reduce to [0, q)
                    u64 u = shoup_lazy(U, pi.ninv, pi.ninvp, q);
                    u64 v = shoup_lazy(D, pi.ninvw1, pi.ninvw1p, q);
                    s[r0 * C + c] = u >= q ? u - q : u;
                    s[r1 * C + c] = v >= q ? v - q : v;
                }
            }
            __syncthreads();
        }
        for (int idx = tid; idx < N1 * C; idx += kThreads) {
            int r = idx / C, c = idx - r * C;
            a[(size_t)r * N2 + c0 + c] = s[idx];
        }
    }
}

// ---------------------------------------------------------------- pass B
// One workgroup: R consecutive rows (N2 contiguous words each) of one limb.
template <int LOGN2, bool INVERSE>
__global__ void __launch_bounds__(kThreads) ntt_pass_rows(LimbSet ls, const u64 *__restrict__ tw,
                                                          const PrimeInfo *__restrict__ pinfo, int logN) {
    constexpr int N2 = 1 << LOGN2;
    __shared__ u64 s[kLdsWords];
    const int N = 1 << logN, N1 = N >> LOGN2;
    const int R = min(kLdsWords / N2, N1);
    const int rowblocks = N1 / R;
    const int job = blockIdx.x / rowblocks, u0 = (blockIdx.x - job * rowblocks) * R;
    int prime;
    u64 *a = limb_ptr(ls, job, N, prime) + (size_t)u0 * N2;
    const u64 q = pinfo[prime].q, q2 = 2 * q;
    const Tw t = tables(tw, prime, N);
    const int tid = threadIdx.x;

    for (int idx = tid; idx < R * N2; idx += kThreads) s[idx] = a[idx];
    __syncthreads();

    if (!INVERSE) {
        for (int ml = 1, h = N2 / 2; ml < N2; ml <<= 1, h >>= 1) {
            const int mg = ml * N1;
            for (int bf = tid; bf < R * N2 / 2; bf += kThreads) {
                int rr = bf / (N2 / 2), k = bf - rr * (N2 / 2);
                int i = k / h, j = k - i * h;
                int x0 = rr * N2 + 2 * i * h + j, x1 = x0 + h;
                int wi = mg + (u0 + rr) * ml + i;
                u64 X = s[x0], Y = s[x1];
                X = X >= q2 ? X - q2 : X;
                u64 T = shoup_lazy(Y, t.W[wi], t.Wp[wi], q);
                s[x0] = X + T;
                s[x1] = X - T + q2;
            }
            __syncthreads();
        }
        for (int idx = tid; idx < R * N2; idx += kThreads) {
            u64 x = s[idx];
            x = x >= q2 ? x - q2 : x;
            a[idx] = x >= q ? x - q : x;
        }
    } else {
        for (int ml = N2 / 2, h = 1; ml >= 1; ml >>= 1, h <<= 1) {
            const int mg = ml * N1;
            for (int bf = tid; bf < R * N2 / 2; bf += kThreads) {
                int rr = bf / (N2 / 2), k = bf - rr * (N2 / 2);
                int i = k / h, j = k - i * h;
                int x0 = rr * N2 + 2 * i * h + j, x1 = x0 + h;
                int wi = mg + (u0 + rr) * ml + i;
                u64 X = s[x0], Y = s[x1];
                u64 U = X + Y;
                U = U >= q2 ? U - q2 : U;
                s[x0] = U;
                s[x1] = shoup_lazy(X - Y + q2, t.Wi[wi], t.Wip[wi], q);
            }
            __syncthreads();
        }
        for (int idx = tid; idx < R * N2; idx += kThreads) a[idx] = s[idx];
    }
}

template <bool INVERSE>
void launch_cols(int logN1, int logN, const LimbSet &ls, const bc_ctx *c, hipStream_t st) {
    int N2 = 1 << (logN - logN1), C = ((16 << logN1) <= kLdsWords) ? 16 : (kLdsWords >> logN1);
    int njobs = ls.npoly * ls.nlimb;
    dim3 grid((unsigned)(njobs * (N2 / C)));
#define BC_COLS(L)                                                                                \
    case L:                                                                                       \
        ntt_pass_cols<L, INVERSE><<<grid, kThreads, 0, st>>>(ls, c->tw, c->pinfo, logN);          \
        break;
    switch (logN1) {
        BC_COLS(5) BC_COLS(6) BC_COLS(7) BC_COLS(8)
        default: throw Error(BC_ERR_PARAM, "ntt: unsupported column length");
    }
#undef BC_COLS
}

template <bool INVERSE>
void launch_rows(int logN2, int logN, const LimbSet &ls, const bc_ctx *c, hipStream_t st) {
    int N1 = 1 << (logN - logN2), R = std::min(kLdsWords >> logN2, N1);
    int njobs = ls.npoly * ls.nlimb;
    dim3 grid((unsigned)(njobs * (N1 / R)));
#define BC_ROWS(L)                                                                                \
    case L:                                                                                       \
        ntt_pass_rows<L, INVERSE><<<grid, kThreads, 0, st>>>(ls, c->tw, c->pinfo, logN);          \
        break;
    switch (logN2) {
        BC_ROWS(5) BC_ROWS(6) BC_ROWS(7) BC_ROWS(8)
        default: throw Error(BC_ERR_PARAM, "ntt: unsupported row length");
    }
#undef BC_ROWS
}

}  // namespace

// N1 = 2^floor(logN/2) rows, N2 = 2^ceil(logN/2) columns.
// Algorithmic bytes of a transform: every limb read once and written once.
static double ntt_bytes(const bc_ctx *c, const LimbSet &ls) { return 16.0 * c->N * ls.npoly * ls.nlimb; }

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
