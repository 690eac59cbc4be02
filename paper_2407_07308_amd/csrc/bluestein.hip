// bluestein.hip -- coefficients <-> evaluation representation of the rings
// Z_q[X]/(Phi_m(X)), m odd, by Bluestein's method (paper, Background,
// "Efficient Polynomial and NTT": the input multiplied by the chirp TF1,
// zero-padded to a power-of-two length L >= 2m - 1, multiplied by the padded
// chirp polynomial D through power-of-two NTTs, the product truncated to m
// words with the excess added back, multiplied by TF1 again, and filtered
// from m to phi(m) positions).
//
// With omega of order m and psi = omega^((m+1)/2) (so psi^2 = omega, psi^m = 1),
// omega^(jk) = psi^(j^2) psi^(k^2) psi^(-(k-j)^2), hence
//   A_k = psi^(k^2) sum_j (a_j psi^(j^2)) psi^(-(k-j)^2):
// a cyclic convolution of length m (psi^(-t^2) is m-periodic in t), done as a
// linear one of length 2m - 1 on the negacyclic transforms of length L and
// folded (c_k = lin_k + lin_(k+m)).  The evaluation representation keeps the
// positions k prime to m (the primitive roots; Phi_m vanishes exactly there),
// in ascending order; the filter is the paper's branch-free selective copy:
// every position's destination is an exclusive prefix sum of the membership
// mask, computed once on the host (the offline phase), so the online copy is
// one independent thread per position (The Design of BoostCom, "GPU-related
// Optimizations", branch removal).
//
// The inverse runs the same convolution with psi^-1 on the values placed at
// their positions (zeros elsewhere) and scaled by m^-1: a polynomial b of
// degree < m with the given values at the primitive roots and 0 at the
// others, so its remainder modulo Phi_m is the answer.  Phi_m is monic of
// degree n = phi(m): with D = m - n, the quotient h of b by Phi_m satisfies
// rev(h) = rev(b) rev(Phi_m)^-1 mod X^D (reversals at degrees D-1, m-1, n),
// a short product with a series inverse computed once per prime, and the
// remainder is b - h Phi_m on the low n coefficients, h Phi_m (degree m - 1 <
// L) formed on the same length-L transforms with Phi_m's transform computed
// once per prime.
//
// Plan reuse (same section: plan reuse for BluesteinFFT): primes, roots,
// chirps, the transformed chirp polynomials, the mask and its prefix sum, the
// series inverse and Phi_m are built once per plan.

#include "bluestein.h"
#include "kernels.h"
#include "ops.h"
#include "persist.h"

#include <algorithm>
#include <cmath>
#include <memory>
#include <numeric>

struct bc_bluestein {
    int m = 0, n = 0, L = 0, logL = 0, D = 0, np = 0;
    std::vector<bc::u64> mod;
    bc_ctx *nt = nullptr;  // power-of-two transform context of length L over the plan's primes
    // device tables, [np][len][2] pairs (value, Shoup companion)
    bc::u64 *tf = nullptr, *tfi = nullptr, *tfis = nullptr, *dh = nullptr, *dih = nullptr, *rinv = nullptr;
    bc::u64 *phih = nullptr;  // transform of Phi_m zero-padded to L
    uint8_t *inz = nullptr;
    int *sumz = nullptr;
    ~bc_bluestein();
};

namespace bc {

namespace {

constexpr int kBT = 256;

// C_pad[ct][i][j] = a_j psi_i^(j^2) for j < n, 0 for n <= j < L
__global__ void k_bs_chirp_pad(const u64 *__restrict__ in, u64 *__restrict__ W, const u64 *__restrict__ tf,
                               const PrimeInfo *__restrict__ pinfo, int n, int m, int L, int np) {
    const int j = blockIdx.x * kBT + threadIdx.x, i = blockIdx.y, ct = blockIdx.z;
    if (j >= L) return;
    u64 v = 0;
    if (j < n) {
        const u64 *t = tf + ((size_t)i * m + j) * 2;
        v = shoup(in[((size_t)ct * np + i) * n + j], t[0], t[1], pinfo[i].q);
    }
    W[((size_t)ct * np + i) * L + j] = v;
}

// inverse: B_pad[ct][i][j] = A_(pos j) psi_i^(-j^2) for j < m prime to m, else 0
__global__ void k_bs_unfilter_chirp(const u64 *__restrict__ in, u64 *__restrict__ W, const u64 *__restrict__ tfi,
                                    const uint8_t *__restrict__ inz, const int *__restrict__ sumz,
                                    const PrimeInfo *__restrict__ pinfo, int n, int m, int L, int np) {
    const int j = blockIdx.x * kBT + threadIdx.x, i = blockIdx.y, ct = blockIdx.z;
    if (j >= L) return;
    u64 v = 0;
    if (j < m && inz[j]) {
        const u64 *t = tfi + ((size_t)i * m + j) * 2;
        v = shoup(in[((size_t)ct * np + i) * n + sumz[j]], t[0], t[1], pinfo[i].q);
    }
    W[((size_t)ct * np + i) * L + j] = v;
}

// W[ct][i][j] *= T[i][j] (the transformed chirp polynomial)
__global__ void k_bs_pointwise(u64 *__restrict__ W, const u64 *__restrict__ T, const PrimeInfo *__restrict__ pinfo,
                               int L, int np) {
    const int j = blockIdx.x * kBT + threadIdx.x, i = blockIdx.y, ct = blockIdx.z;
    if (j >= L) return;
    const u64 *t = T + ((size_t)i * L + j) * 2;
    u64 &w = W[((size_t)ct * np + i) * L + j];
    w = shoup(w, t[0], t[1], pinfo[i].q);
}

// forward: out[ct][i][sumz[k]] = (lin_k + lin_(k+m)) psi_i^(k^2) for k < m prime to m
__global__ void k_bs_fold_filter(const u64 *__restrict__ W, u64 *__restrict__ out, const u64 *__restrict__ tf,
                                 const uint8_t *__restrict__ inz, const int *__restrict__ sumz,
                                 const PrimeInfo *__restrict__ pinfo, int n, int m, int L, int np) {
    const int k = blockIdx.x * kBT + threadIdx.x, i = blockIdx.y, ct = blockIdx.z;
    if (k >= m || !inz[k]) return;
    const u64 q = pinfo[i].q;
    const u64 *w = W + ((size_t)ct * np + i) * L;
    const u64 *t = tf + ((size_t)i * m + k) * 2;
    out[((size_t)ct * np + i) * n + sumz[k]] = shoup(add_mod(w[k], w[k + m], q), t[0], t[1], q);
}

// inverse: b_j = (lin_j + lin_(j+m)) psi_i^(-j^2) m^-1 for j < m, in place
// (thread j reads words j and j + m and writes word j only)
__global__ void k_bs_fold_chirp(u64 *__restrict__ W, const u64 *__restrict__ tfis, const PrimeInfo *__restrict__ pinfo,
                                int m, int L, int np) {
    const int j = blockIdx.x * kBT + threadIdx.x, i = blockIdx.y, ct = blockIdx.z;
    if (j >= m) return;
    const u64 q = pinfo[i].q;
    u64 *w = W + ((size_t)ct * np + i) * L;
    const u64 *t = tfis + ((size_t)i * m + j) * 2;
    w[j] = shoup(add_mod(w[j], w[j + m], q), t[0], t[1], q);
}

// quotient of b (W[.][.][0..m)) by Phi_m, zero-padded to L: for s < D,
// rev(h)_s = sum_(u <= s) b_(m-1-u) rinv_(s-u) goes to position D-1-s;
// positions D .. L-1 are zero
__global__ void k_bs_quotient(const u64 *__restrict__ W, u64 *__restrict__ H, const u64 *__restrict__ rinv,
                              const PrimeInfo *__restrict__ pinfo, int m, int D, int L, int np) {
    const int s = blockIdx.x * kBT + threadIdx.x, i = blockIdx.y, ct = blockIdx.z;
    if (s >= L) return;
    u64 *hrow = H + ((size_t)ct * np + i) * L;
    if (s >= D) {
        hrow[s] = 0;
        return;
    }
    const u64 q = pinfo[i].q;
    const u64 *b = W + ((size_t)ct * np + i) * L;
    const u64 *r = rinv + (size_t)i * D * 2;
    u64 acc = 0;
    for (int u = 0; u <= s; u++) acc = add_mod(acc, shoup(b[m - 1 - u], r[2 * (s - u)], r[2 * (s - u) + 1], q), q);
    hrow[D - 1 - s] = acc;
}

// a_j = b_j - (h Phi_m)_j, j < n
__global__ void k_bs_remainder(const u64 *__restrict__ W, const u64 *__restrict__ HP, u64 *__restrict__ out,
                               const PrimeInfo *__restrict__ pinfo, int n, int L, int np) {
    const int j = blockIdx.x * kBT + threadIdx.x, i = blockIdx.y, ct = blockIdx.z;
    if (j >= n) return;
    const size_t row = ((size_t)ct * np + i) * L;
    out[((size_t)ct * np + i) * n + j] = sub_mod(W[row + j], HP[row + j], pinfo[i].q);
}

dim3 grid_of(int len, int np, int count) { return dim3((unsigned)((len + kBT - 1) / kBT), (unsigned)np, (unsigned)count); }

// Phi_m by recursion over the divisors: Phi_d = (X^d - 1) / prod_(e | d, e < d) Phi_e
std::vector<int64_t> cyclotomic_poly(int m) {
    std::vector<int> divs;
    for (int d = 1; d <= m; d++)
        if (m % d == 0) divs.push_back(d);
    std::vector<std::vector<int64_t>> ph(divs.size());
    for (size_t a = 0; a < divs.size(); a++) {
        const int d = divs[a];
        std::vector<int64_t> den{1};
        for (size_t b = 0; b < a; b++) {
            if (d % divs[b]) continue;
            std::vector<int64_t> pr(den.size() + ph[b].size() - 1, 0);
            for (size_t x = 0; x < den.size(); x++)
                for (size_t y = 0; y < ph[b].size(); y++) pr[x + y] += den[x] * ph[b][y];
            den = pr;
        }
        // (X^d - 1) / den, den monic of degree e: long division from the top
        std::vector<int64_t> num(d + 1, 0);
        num[0] = -1;
        num[d] = 1;
        const int e = (int)den.size() - 1, qd = d - e;
        std::vector<int64_t> quo(qd + 1, 0);
        for (int t = d; t >= e; t--) {
            const int64_t c = num[t];
            quo[t - e] = c;
            if (c)
                for (int x = 0; x <= e; x++) num[t - e + x] -= c * den[x];
        }
        for (int x = 0; x < e; x++) BC_REQUIRE(num[x] == 0, BC_ERR_PARAM, "cyclotomic division left a remainder");
        ph[a] = quo;
    }
    return ph.back();
}

// smallest x >= 2 with x^((q-1)/m) of order exactly m
u64 order_m_root(u64 q, u64 m) {
    std::vector<u64> fac;
    u64 t = m;
    for (u64 r = 2; r * r <= t; r++)
        if (t % r == 0) {
            fac.push_back(r);
            while (t % r == 0) t /= r;
        }
    if (t > 1) fac.push_back(t);
    for (u64 x = 2; x < q; x++) {
        const u64 w = h_powmod(x, (q - 1) / m, q);
        bool ok = w != 1;
        for (u64 f : fac) ok = ok && h_powmod(w, m / f, q) != 1;
        if (ok) return w;
    }
    throw Error(BC_ERR_PARAM, "no root of unity of order m");
}

template <class T>
T *upload_vec(const std::vector<T> &h) {
    T *d = nullptr;
    BC_HIP(hipMalloc(&d, sizeof(T) * std::max<size_t>(1, h.size())));
    if (!h.empty()) BC_HIP(hipMemcpy(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
    return d;
}

void push_pair(std::vector<u64> &v, u64 w, u64 q) {
    v.push_back(w);
    v.push_back(h_shoup(w, q));
}

// the plan's primes as one limb set of `count` polynomials [count][np][L]
LimbSet plan_limbs(const bc_bluestein *b, u64 *base, int count) {
    LimbSet ls{};
    ls.base = base;
    ls.poly_stride = (u64)b->np * b->L;
    ls.npoly = count;
    ls.nlimb = b->np;
    for (int k = 0; k < b->np; k++) {
        ls.off[k] = (int16_t)k;
        ls.prime[k] = (int16_t)k;
    }
    return ls;
}

// The convolution: NTT of W, product with T, inverse NTT (in place).
void convolve(bc_bluestein *b, u64 *W, const u64 *T, int count, hipStream_t st) {
    const LimbSet ls = plan_limbs(b, W, count);
    ntt_forward(b->nt, ls, st);
    k_bs_pointwise<<<grid_of(b->L, b->np, count), kBT, 0, st>>>(W, T, b->nt->pinfo, b->L, b->np);
    BC_HIP(hipGetLastError());
    ntt_inverse(b->nt, ls, st);
}

struct StreamTag {
    hipStream_t prev;
    explicit StreamTag(hipStream_t s) : prev(tl_stream) { tl_stream = s; }
    ~StreamTag() { tl_stream = prev; }
};

}  // namespace

bc_bluestein *bluestein_create(int m, int np, int bits) {
    BC_REQUIRE(m >= 3 && (m & 1) && m <= 32767, BC_ERR_PARAM, "m must be odd, in [3, 32767]");
    BC_REQUIRE(np >= 1 && np + 1 <= kMaxMod && np <= kMaxJobs, BC_ERR_PARAM, "bad prime count");
    BC_REQUIRE(bits >= 30 && bits <= 61, BC_ERR_PARAM, "prime size must be in [30, 61] bits");
    std::unique_ptr<bc_bluestein> b(new bc_bluestein());
    b->m = m;
    int logL = 10;
    while ((1 << logL) < 2 * m - 1) logL++;
    BC_REQUIRE(logL <= 16, BC_ERR_PARAM, "the convolution length exceeds 2^16");
    b->logL = logL;
    b->L = 1 << logL;
    b->np = np;
    const std::vector<int64_t> phi = cyclotomic_poly(m);
    b->n = (int)phi.size() - 1;
    b->D = m - b->n;
    // primes 1 mod 2 L m (m-th roots, negacyclic transforms of length L); one
    // more serves as the transform context's unused special prime
    const u64 step = 2 * (u64)b->L * (u64)m;
    std::vector<u64> pr = primes_one_mod(step, bits, np + 1);
    b->mod.assign(pr.begin(), pr.begin() + np);
    bc_params prm{logL, 3, np, bits, 1, bits, np};
    b->nt = new bc_ctx();
    build_context_moduli(b->nt, prm, pr);

    const int L = b->L, n = b->n, D = b->D;
    // the mask of positions prime to m and its exclusive prefix sum (offline phase)
    std::vector<uint8_t> inz(m);
    std::vector<int> sumz(m);
    int run = 0;
    for (int k = 0; k < m; k++) {
        inz[k] = std::gcd(k, m) == 1;
        sumz[k] = run;
        run += inz[k];
    }
    BC_REQUIRE(run == n, BC_ERR_PARAM, "phi(m) and the cyclotomic degree disagree");
    std::vector<u64> tf, tfi, tfis, dpad((size_t)np * L, 0), dipad((size_t)np * L, 0), phpad((size_t)np * L, 0), rinv;
    for (int i = 0; i < np; i++) {
        const u64 q = b->mod[i];
        const u64 w = order_m_root(q, (u64)m), psi = h_powmod(w, (u64)(m + 1) / 2, q);
        const u64 ipsi = h_invmod(psi, q), minv = h_invmod((u64)m % q, q);
        std::vector<u64> pp(m), ip(m);  // psi^e, psi^-e for e < m
        pp[0] = ip[0] = 1;
        for (int e = 1; e < m; e++) {
            pp[e] = h_mulmod(pp[e - 1], psi, q);
            ip[e] = h_mulmod(ip[e - 1], ipsi, q);
        }
        for (int j = 0; j < m; j++) {
            const int e = (int)((int64_t)j * j % m);
            push_pair(tf, pp[e], q);
            push_pair(tfi, ip[e], q);
            push_pair(tfis, h_mulmod(ip[e], minv, q), q);
            dpad[(size_t)i * L + j] = ip[e];
            dipad[(size_t)i * L + j] = pp[e];
        }
        // series inverse of rev(Phi_m) = sum_j Phi_(n-j) X^j (constant term 1) mod X^D
        std::vector<u64> rv(D), rp(n + 1);
        for (int j = 0; j <= n; j++) {
            const int64_t c = phi[n - j];
            rp[j] = c >= 0 ? (u64)c % q : q - (u64)(-c) % q;
        }
        for (int s = 0; s < D; s++) {
            u64 acc = s == 0 ? 1 : 0;
            for (int j = 1; j <= std::min(s, n); j++) acc = (acc + q - h_mulmod(rp[j], rv[s - j], q)) % q;
            rv[s] = acc;
        }
        for (int s = 0; s < D; s++) push_pair(rinv, rv[s], q);
        for (int j = 0; j <= n; j++) phpad[(size_t)i * L + j] = rp[n - j];
    }
    b->tf = upload_vec(tf);
    b->tfi = upload_vec(tfi);
    b->tfis = upload_vec(tfis);
    b->rinv = upload_vec(rinv);
    b->inz = upload_vec(inz);
    b->sumz = upload_vec(sumz);
    // the transformed chirp polynomials and Phi_m (once per plan), with Shoup
    // companions
    for (int pass = 0; pass < 3; pass++) {
        std::vector<u64> &h = pass == 2 ? phpad : pass ? dipad : dpad;
        u64 *d = upload_vec(h);
        ntt_forward(b->nt, plan_limbs(b.get(), d, 1), nullptr);
        BC_HIP(hipMemcpy(h.data(), d, sizeof(u64) * h.size(), hipMemcpyDeviceToHost));
        BC_HIP(hipFree(d));
        std::vector<u64> pairs;
        pairs.reserve(2 * h.size());
        for (int i = 0; i < np; i++)
            for (int j = 0; j < L; j++) push_pair(pairs, h[(size_t)i * L + j], b->mod[i]);
        (pass == 2 ? b->phih : pass ? b->dih : b->dh) = upload_vec(pairs);
    }
    return b.release();
}

void bluestein_destroy(bc_bluestein *b) { delete b; }

void bluestein_info(const bc_bluestein *b, int *n, int *conv_len, u64 *moduli) {
    if (n) *n = b->n;
    if (conv_len) *conv_len = b->L;
    if (moduli) std::copy(b->mod.begin(), b->mod.end(), moduli);
}

void bluestein_forward(bc_bluestein *b, const u64 *in, u64 *out, int count, hipStream_t st) {
    BC_REQUIRE(count >= 1 && count <= 65535 && in && out, BC_ERR_ARG, "bad batch");
    StreamTag tag(st);
    BufP W = make_buf(b->nt, sizeof(u64) * (size_t)count * b->np * b->L);
    u64 *w = (u64 *)W->p;
    const PrimeInfo *pi = b->nt->pinfo;
    k_bs_chirp_pad<<<grid_of(b->L, b->np, count), kBT, 0, st>>>(in, w, b->tf, pi, b->n, b->m, b->L, b->np);
    BC_HIP(hipGetLastError());
    convolve(b, w, b->dh, count, st);
    k_bs_fold_filter<<<grid_of(b->m, b->np, count), kBT, 0, st>>>(w, out, b->tf, b->inz, b->sumz, pi, b->n, b->m,
                                                                  b->L, b->np);
    BC_HIP(hipGetLastError());
}

void bluestein_inverse(bc_bluestein *b, const u64 *in, u64 *out, int count, hipStream_t st) {
    BC_REQUIRE(count >= 1 && count <= 65535 && in && out, BC_ERR_ARG, "bad batch");
    StreamTag tag(st);
    BufP W = make_buf(b->nt, sizeof(u64) * (size_t)count * b->np * b->L);
    BufP H = make_buf(b->nt, sizeof(u64) * (size_t)count * b->np * b->L);
    u64 *w = (u64 *)W->p, *h = (u64 *)H->p;
    const PrimeInfo *pi = b->nt->pinfo;
    k_bs_unfilter_chirp<<<grid_of(b->L, b->np, count), kBT, 0, st>>>(in, w, b->tfi, b->inz, b->sumz, pi, b->n, b->m,
                                                                     b->L, b->np);
    BC_HIP(hipGetLastError());
    convolve(b, w, b->dih, count, st);
    k_bs_fold_chirp<<<grid_of(b->m, b->np, count), kBT, 0, st>>>(w, b->tfis, pi, b->m, b->L, b->np);
    k_bs_quotient<<<grid_of(b->L, b->np, count), kBT, 0, st>>>(w, h, b->rinv, pi, b->m, b->D, b->L, b->np);
    BC_HIP(hipGetLastError());
    convolve(b, h, b->phih, count, st);  // h Phi_m
    k_bs_remainder<<<grid_of(b->n, b->np, count), kBT, 0, st>>>(w, h, out, pi, b->n, b->L, b->np);
    BC_HIP(hipGetLastError());
}

}  // namespace bc

bc_bluestein::~bc_bluestein() {
    (void)hipDeviceSynchronize();
    for (void *p : {(void *)tf, (void *)tfi, (void *)tfis, (void *)dh, (void *)dih, (void *)rinv, (void *)phih,
                    (void *)inz, (void *)sumz})
        if (p) (void)hipFree(p);
    delete nt;
}
