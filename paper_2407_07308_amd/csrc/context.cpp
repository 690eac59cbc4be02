// context.cpp -- parameter set, prime chain and every precomputed table.
//
// All tables are built once per context and kept in HBM (the device-side
// analogue of the paper's plan reuse, "GPU-related Optimizations": work that
// does not depend on the data leaves the critical path).

#include <algorithm>
#include <cstring>

#include "ops.h"
#include "persist.h"

namespace bc {

u64 h_mulmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }

u64 h_powmod(u64 b, u64 e, u64 q) {
    u64 r = 1 % q;
    b %= q;
    for (; e; e >>= 1) {
        if (e & 1) r = h_mulmod(r, b, q);
        b = h_mulmod(b, b, q);
    }
    return r;
}

u64 h_invmod(u64 a, u64 q) {
    // extended Euclid on signed 128-bit values
    __int128 t = 0, nt = 1, r = q, nr = a % q;
    while (nr != 0) {
        __int128 k = r / nr, tmp = t - k * nt;
        t = nt;
        nt = tmp;
        tmp = r - k * nr;
        r = nr;
        nr = tmp;
    }
    if (t < 0) t += q;
    return (u64)t;
}

int bit_reverse(int x, int bits) {
    int r = 0;
    for (int i = 0; i < bits; i++) r |= ((x >> i) & 1) << (bits - 1 - i);
    return r;
}

namespace {

// Miller-Rabin with the seven bases of J. Sinclair, deterministic for n < 2^64.
bool is_prime64(u64 n) {
    if (n < 4) return n >= 2;
    if (n % 2 == 0) return false;
    u64 d = n - 1;
    int s = __builtin_ctzll(d);
    d >>= s;
    static const u64 bases[] = {2, 325, 9375, 28178, 450775, 9780504, 1795265022};
    for (u64 a : bases) {
        a %= n;
        if (a == 0) continue;
        u64 x = h_powmod(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool witness = true;
        for (int r = 1; r < s && witness; r++) {
            x = h_mulmod(x, x, n);
            if (x == n - 1) witness = false;
        }
        if (witness) return false;
    }
    return true;
}

// Largest `count` primes p < 2^bits with p = 1 mod step, skipping `taken`.
std::vector<u64> prime_chain(u64 step, int bits, int count, const std::vector<u64> &taken) {
    std::vector<u64> out;
    u64 limit = (bits >= 64) ? ~(u64)0 : ((u64)1 << bits);
    u64 k = (limit - 2) / step;
    for (; k > 0 && (int)out.size() < count; k--) {
        u64 c = k * step + 1;
        if (std::find(taken.begin(), taken.end(), c) != taken.end()) continue;
        if (is_prime64(c)) out.push_back(c);
    }
    if ((int)out.size() != count) throw Error(BC_ERR_PARAM, "not enough primes of the requested size");
    return out;
}

// Primitive 2N-th root of unity: g^((q-1)/2N) for a generator g of Z_q^*.
u64 root_2n(u64 q, int N) {
    u64 phi = q - 1, n = phi;
    std::vector<u64> fac;
    for (u64 f = 2; f * f <= n; f += (f == 2 ? 1 : 2))
        if (n % f == 0) {
            fac.push_back(f);
            while (n % f == 0) n /= f;
        }
    if (n > 1) fac.push_back(n);
    for (u64 g = 2;; g++) {
        bool gen = true;
        for (u64 f : fac)
            if (h_powmod(g, phi / f, q) == 1) { gen = false; break; }
        if (gen) return h_powmod(g, phi / (2 * (u64)N), q);
    }
}

template <class T>
T *upload(const T *h, size_t n) {
    T *d = nullptr;
    BC_HIP(hipMalloc(&d, sizeof(T) * n));
    BC_HIP(hipMemcpy(d, h, sizeof(T) * n, hipMemcpyHostToDevice));
    return d;
}

void set_shoup(u64 dst[2], u64 w, u64 q) {
    dst[0] = w % q;
    dst[1] = h_shoup(dst[0], q);
}

void set_fpair(u64 dst[2], u64 w, u64 q) { h_fpair(dst, w, q); }

// Tables of the matrix-core modulus raising (b_modup_mfma): for PL folded
// forward stages (NV = 2^PL words per base position), plan (level, digit),
// target t and output word v, the row block of M[t][v][s][v'] 2^(8a) mod p_t
// as seven signed base-256 digits, K = (s NV + v') 8 + a, and the correction
// 128 sum_K W mod p_t.  Built when every digit fits the kernel (alpha NV <= 32)
// and every prime exceeds 2^33 (2^32 is its own residue in the recombination).
void build_modup_mfma(bc_ctx *c) {
    const int nm = c->nmod, nplans = (int)c->h_modup.size();
    for (int m = 0; m < nm; m++)
        if (c->mod[m] <= ((u64)1 << 33)) return;
    for (int PL = 0; PL <= 2; PL++) {
        const int NV = 1 << PL, TPT = 4 / NV;
        if (c->alpha * NV > 32 || (c->N >> PL) % 128) continue;
        const int kpad = 32 * ((c->alpha * NV * 8 + 31) / 32);
        const int tiles = (nm + TPT - 1) / TPT, stride = tiles * 32 * kpad;
        std::vector<int8_t> w((size_t)nplans * stride, 0);
        std::vector<double> corr((size_t)nplans * nm * 4, 0.0);
        for (int pi = 0; pi < nplans; pi++) {
            const ModUpPlan &pl = c->h_modup[pi];
            for (int t = 0; t < pl.ntgt; t++) {
                const int pm = pl.tgt_prime[t];
                const u64 q = c->mod[pm];
                const u64 w1 = c->h_pinfo[pm].w123[0][0], w2 = c->h_pinfo[pm].w123[1][0],
                          w3 = c->h_pinfo[pm].w123[2][0];
                // the fold's matrix: out[v] = sum_v' F[v][v'] in[v'] (the forward stages of fold_fp)
                u64 F[4][4] = {{1}};
                if (PL == 1) {
                    F[0][0] = 1, F[0][1] = w1, F[1][0] = 1, F[1][1] = q - w1;
                } else if (PL == 2) {
                    const u64 w21 = h_mulmod(w2, w1, q), w31 = h_mulmod(w3, w1, q);
                    const u64 rows[4][4] = {{1, w2, w1, w21},
                                            {1, q - w2, w1, (q - w21) % q},
                                            {1, w3, q - w1, (q - w31) % q},
                                            {1, q - w3, q - w1, w31}};
                    std::memcpy(F, rows, sizeof(F));
                }
                for (int v = 0; v < NV; v++) {
                    const int unit = (t % TPT) * NV + v, h = unit / 2;
                    int8_t *blk = &w[(size_t)pi * stride + (size_t)(t / TPT) * 32 * kpad];
                    u64 csum = 0;
                    for (int sidx = 0; sidx < pl.nsrc; sidx++)
                        for (int v2 = 0; v2 < NV; v2++) {
                            u64 W = h_mulmod(F[v][v2], pl.qhat[t][sidx][0], q);
                            for (int a = 0; a < 7; a++, W = h_mulmod(W, 256, q)) {
                                csum = (csum + W) % q;
                                int64_t x = (int64_t)W;
                                const int K = (sidx * NV + v2) * 8 + a;
                                for (int b = 0; b < 7; b++) {
                                    int64_t d = x & 255;
                                    if (d >= 128) d -= 256;
                                    x = (x - d) / 256;
                                    const int r = 8 * (unit % 2) + b, row = 8 * (r / 4) + 4 * h + r % 4;
                                    blk[(size_t)row * kpad + K] = (int8_t)d;
                                }
                                BC_REQUIRE(x == 0, BC_ERR_PARAM, "modulus raising weight beyond seven digits");
                            }
                        }
                    corr[((size_t)pi * nm + t) * 4 + v] = (double)h_mulmod(csum, 128, q);
                }
            }
        }
        ModUpMfma &T = c->modup_mfma[PL];
        T.w8 = upload(w.data(), w.size());
        T.corr = upload(corr.data(), corr.size());
        T.kpad = kpad;
        T.plan_stride = stride;
    }
}

typedef void (*PairSet)(u64 dst[2], u64 w, u64 q);

// Base-conversion and modulus-switching constants, each stored as a pair by
// `setp` (Shoup pairs for the integer kernels, FPairs for the fp64 ones).
void build_plans(const bc_ctx *c, PairSet setp, std::vector<ModUpPlan> &mu, ModDownPlan &md,
                 std::vector<ModSwitchPlan> &ms) {
    const int nQ = c->nQ, nP = c->nP;
    // modulus raising, one plan per (level, digit)
    mu.assign((size_t)nQ * c->dnum, ModUpPlan{});
    for (int lv = 0; lv < nQ; lv++)
        for (int j = 0; j < c->dnum; j++) {
            ModUpPlan &pl = mu[(size_t)lv * c->dnum + j];
            int lo = j * c->alpha, hi = std::min(std::min((j + 1) * c->alpha, nQ), lv + 1);
            pl.src_lo = lo;
            pl.nsrc = std::max(0, hi - lo);
            pl.ntgt = 0;
            if (pl.nsrc == 0) continue;
            for (int i = lo; i < hi; i++) {
                u64 q = c->mod[i], prod = 1;
                for (int t = lo; t < hi; t++)
                    if (t != i) prod = h_mulmod(prod, c->mod[t] % q, q);
                setp(pl.qhinv[i - lo], h_invmod(prod, q), q);
            }
            int next = lv + 1 + nP;
            for (int e = 0; e < next; e++) {
                if (e >= lo && e < hi) continue;
                int prime = e <= lv ? e : nQ + (e - lv - 1);
                u64 q = c->mod[prime];
                int t = pl.ntgt++;
                pl.tgt_e[t] = e;
                pl.tgt_prime[t] = prime;
                for (int i = lo; i < hi; i++) {
                    u64 prod = 1;
                    for (int k = lo; k < hi; k++)
                        if (k != i) prod = h_mulmod(prod, c->mod[k] % q, q);
                    setp(pl.qhat[t][i - lo], prod, q);
                }
            }
        }
    // modulus lowering (exact division by P)
    std::memset(&md, 0, sizeof(ModDownPlan));
    for (int j = 0; j < nP; j++) {
        u64 pj = c->mod[nQ + j], prod = 1;
        for (int t = 0; t < nP; t++)
            if (t != j) prod = h_mulmod(prod, c->mod[nQ + t] % pj, pj);
        setp(md.vfac[j], h_mulmod(h_invmod(c->p % pj, pj), h_invmod(prod, pj), pj), pj);
    }
    for (int i = 0; i < nQ; i++) {
        u64 q = c->mod[i], P = 1;
        for (int j = 0; j < nP; j++) {
            u64 prod = 1;
            for (int t = 0; t < nP; t++)
                if (t != j) prod = h_mulmod(prod, c->mod[nQ + t] % q, q);
            setp(md.phat[i][j], prod, q);
            P = h_mulmod(P, c->mod[nQ + j] % q, q);
        }
        u64 Pinv = h_invmod(P, q);
        setp(md.pinv[i], Pinv, q);
        const u64 ppi = h_mulmod(Pinv, c->p % q, q);
        setp(md.ppinv[i], ppi, q);
        for (int j = 0; j < nP; j++) {
            u64 prod = 1;
            for (int t = 0; t < nP; t++)
                if (t != j) prod = h_mulmod(prod, c->mod[nQ + t] % q, q);
            setp(md.phatpp[i][j], h_mulmod(prod, ppi, q), q);
        }
    }
    // modulus switching, one plan per level
    ms.assign(nQ, ModSwitchPlan{});
    std::memset(ms.data(), 0, sizeof(ModSwitchPlan) * nQ);
    for (int lv = 1; lv < nQ; lv++) {
        u64 ql = c->mod[lv];
        ms[lv].ql = ql;
        setp(ms[lv].pinv_l, h_invmod(c->p % ql, ql), ql);
        for (int i = 0; i < lv; i++) {
            const u64 q = c->mod[i], qlinv = h_invmod(ql % q, q);
            setp(ms[lv].qlinv[i], qlinv, q);
            u64 P = 1;
            for (int t = 0; t < nP; t++) P = h_mulmod(P, c->mod[nQ + t] % q, q);
            const u64 ppq = h_mulmod(h_mulmod(c->p % q, h_invmod(P, q), q), qlinv, q);  // p P^-1 q_l^-1
            for (int j = 0; j < nP; j++) {
                u64 phat = 1;
                for (int t = 0; t < nP; t++)
                    if (t != j) phat = h_mulmod(phat, c->mod[nQ + t] % q, q);
                setp(ms[lv].rk1[i][j], h_mulmod(phat, ppq, q), q);
            }
            setp(ms[lv].rk2[i], h_mulmod(c->p % q, qlinv, q), q);
        }
    }
}

}  // namespace

// ------------------------------------------------------------------ pool

thread_local hipStream_t tl_stream = nullptr;
thread_local Arena *tl_arena = nullptr;

// Block sizes are rounded up to a size class (four per power of two, at
// least 256 bytes), and a request takes any cached block of its stream up to
// twice its class (any larger one once the pool is at its limit): batches of
// varying shape then reuse each other's blocks instead of allocating (and
// eventually freeing, which waits for the device).
size_t Pool::size_class(size_t bytes) {
    bytes = std::max<size_t>(bytes, 256);
    int e = 63 - __builtin_clzll(bytes);
    if (e < 2) return 256;
    const size_t step = (size_t)1 << (e - 2);
    return (bytes + step - 1) / step * step;
}

void *Pool::alloc(size_t bytes) {
    bytes = size_class(bytes);
    std::lock_guard<std::mutex> g(mu);
    const hipStream_t st = tl_stream;
    auto it = free_.lower_bound({st, bytes});
    // at the limit, any larger cached block of the stream serves rather than
    // a new one (which would first evict the blocks of other shapes)
    const bool full = limit && held + bytes > limit && !recording;
    if (it != free_.end() && it->first.first == st && (full || it->first.second <= 2 * bytes)) {
        void *p = it->second.p;
        live_[p] = {it->first.second, st};
        cached -= it->first.second;
        free_.erase(it);
        if (recording) recorded.push_back(p);
        return p;
    }
    void *p = nullptr;
    // growing past the limit: give back the cached blocks released longest
    // ago until the new block fits under seven eighths of it (hipFree waits
    // for the device, so blocks whose last users are still queued are safe
    // to free); the blocks of the shapes in current use were released last
    // and stay.  Never while a graph records: it owns the blocks it was handed.
    if (full) evict_to(limit / 8 * 7 > bytes ? limit / 8 * 7 - bytes : 0);
    if (fail_after > 0 && --fail_after == 0) throw Error(BC_ERR_OOM, "device workspace allocation failed (test hook)");
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        // give back every cached block and retry once
        free_cached();
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            throw Error(BC_ERR_OOM, "device workspace allocation failed");
        }
    }
    held += bytes;
    live_[p] = {bytes, st};
    if (recording) recorded.push_back(p);
    return p;
}

std::vector<void *> Pool::detach_recorded() {
    std::lock_guard<std::mutex> g(mu);
    recording = false;
    std::vector<void *> out;
    for (void *p : recorded) {
        if (std::find(out.begin(), out.end(), p) != out.end()) continue;
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second.p == p) {
                held -= it->first.second;
                cached -= it->first.second;
                free_.erase(it);
                out.push_back(p);
                break;
            }
    }
    recorded.clear();
    return out;
}

void Pool::release(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> g(mu);
    auto it = live_.find(p);
    if (it == live_.end()) return;
    free_.emplace(std::make_pair(it->second.second, it->second.first), Cached{p, ++seq});
    cached += it->second.first;
    live_.erase(it);
}

// caller holds mu
void Pool::free_cached() {
    for (auto &kv : free_) {
        (void)hipFree(kv.second.p);
        held -= kv.first.second;
    }
    free_.clear();
    cached = 0;
}

// caller holds mu
void Pool::evict_to(size_t bytes) {
    std::vector<decltype(free_)::iterator> order;
    order.reserve(free_.size());
    for (auto it = free_.begin(); it != free_.end(); ++it) order.push_back(it);
    std::sort(order.begin(), order.end(), [](auto a, auto b) { return a->second.seq < b->second.seq; });
    for (auto it : order) {
        if (held <= bytes) break;
        (void)hipFree(it->second.p);
        held -= it->first.second;
        cached -= it->first.second;
        free_.erase(it);
    }
}

void Pool::trim() {
    std::lock_guard<std::mutex> g(mu);
    free_cached();
}

Pool::~Pool() {
    for (auto &kv : free_) (void)hipFree(kv.second.p);
    for (auto &kv : live_) (void)hipFree(kv.first);
}

// --------------------------------------------------------------- profiler

hipEvent_t Profiler::take() {
    if (!spare.empty()) {
        hipEvent_t e = spare.back();
        spare.pop_back();
        return e;
    }
    hipEvent_t e;
    BC_HIP(hipEventCreate(&e));
    return e;
}

void Profiler::begin(int kind, double bytes, hipStream_t st, ProfRec &r) {
    std::lock_guard<std::mutex> g(mu);
    r.kind = kind;
    r.bytes = bytes;
    r.a = take();
    r.b = take();
    BC_HIP(hipEventRecord(r.a, st));
}

void Profiler::end(ProfRec &r, hipStream_t st) {
    BC_HIP(hipEventRecord(r.b, st));
    std::lock_guard<std::mutex> g(mu);
    recs.push_back(r);
}

void Profiler::clear() {
    std::lock_guard<std::mutex> g(mu);
    for (auto &r : recs) {
        spare.push_back(r.a);
        spare.push_back(r.b);
    }
    recs.clear();
}

Profiler::~Profiler() {
    for (auto &r : recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : spare) (void)hipEventDestroy(e);
}

// ----------------------------------------------------------------- context

std::vector<u64> param_moduli(const bc_params &prm) {
    BC_REQUIRE(prm.logN >= 10 && prm.logN <= 16, BC_ERR_PARAM, "logN must be in [10, 16]");
    BC_REQUIRE(prm.p >= 3 && prm.p < (1 << 20), BC_ERR_PARAM, "p must be a small odd prime");
    BC_REQUIRE(is_prime64((u64)prm.p), BC_ERR_PARAM, "p must be prime");
    BC_REQUIRE(prm.nQ >= 1 && prm.nP >= 1 && prm.nQ + prm.nP <= kMaxMod, BC_ERR_PARAM, "bad prime counts");
    BC_REQUIRE(prm.bitsQ >= 20 && prm.bitsQ <= 61 && prm.bitsP >= 20 && prm.bitsP <= 61, BC_ERR_PARAM,
               "prime sizes must be in [20, 61] bits");
    BC_REQUIRE(prm.dnum >= 1 && prm.dnum <= prm.nQ, BC_ERR_PARAM, "dnum must be in [1, nQ]");
    BC_REQUIRE((prm.nQ + prm.dnum - 1) / prm.dnum <= kMaxDigit && prm.nP <= kMaxDigit, BC_ERR_PARAM,
               "at most 16 primes per digit and 16 special primes");
    const u64 pm1 = (u64)prm.p - 1;
    BC_REQUIRE((1 << (__builtin_ctzll(pm1) - 1)) <= (1 << prm.logN), BC_ERR_PARAM, "more slots than coefficients");
    const u64 step = 2 * ((u64)1 << prm.logN) * (u64)prm.p;
    std::vector<u64> mod = prime_chain(step, prm.bitsQ, prm.nQ, {});
    auto sp = prime_chain(step, prm.bitsP, prm.nP, mod);
    mod.insert(mod.end(), sp.begin(), sp.end());
    return mod;
}

void build_context(bc_ctx *c, const bc_params &prm) { build_context_moduli(c, prm, param_moduli(prm)); }

std::vector<u64> primes_one_mod(u64 step, int bits, int count) { return prime_chain(step, bits, count, {}); }

// A context over explicitly chosen primes (each 1 mod 2N); prm supplies the
// ring degree, the plaintext modulus and the split into nQ + nP primes.
void build_context_moduli(bc_ctx *c, const bc_params &prm, std::vector<u64> mod) {
    BC_REQUIRE((int)mod.size() == prm.nQ + prm.nP && prm.nQ >= 1 && prm.nP >= 1 && (int)mod.size() <= kMaxMod,
               BC_ERR_PARAM, "bad prime counts");
    for (u64 q : mod)
        BC_REQUIRE(q % (2 * ((u64)1 << prm.logN)) == 1 && is_prime64(q), BC_ERR_PARAM,
                   "every prime must be 1 mod 2N");
    c->mod = std::move(mod);
    c->prm = prm;
    c->logN = prm.logN;
    c->N = 1 << prm.logN;
    c->nQ = prm.nQ;
    c->nP = prm.nP;
    c->nmod = prm.nQ + prm.nP;
    c->dnum = prm.dnum;
    c->alpha = (prm.nQ + prm.dnum - 1) / prm.dnum;
    c->p = (u64)prm.p;
    c->M = 1 << (__builtin_ctzll(c->p - 1) - 1);
    c->noise = NoiseModel(prm, c->mod);

    const int N = c->N, nQ = c->nQ, nm = c->nmod;

    // twiddles and per-prime constants
    std::vector<u64> tw((size_t)nm * 4 * N);
    c->h_pinfo.resize(nm);
    for (int m = 0; m < nm; m++) {
        u64 q = c->mod[m];
        u64 psi = root_2n(q, N), ipsi = h_invmod(psi, q);
        u64 *W = &tw[(size_t)m * 4 * N], *Wp = W + N, *Wi = W + 2 * N, *Wip = W + 3 * N;
        std::vector<u64> pw(N), ipw(N);
        pw[0] = ipw[0] = 1;
        for (int k = 1; k < N; k++) {
            pw[k] = h_mulmod(pw[k - 1], psi, q);
            ipw[k] = h_mulmod(ipw[k - 1], ipsi, q);
        }
        for (int k = 0; k < N; k++) {
            int r = bit_reverse(k, c->logN);
            W[k] = pw[r];
            Wi[k] = ipw[r];
            Wp[k] = h_shoup(W[k], q);
            Wip[k] = h_shoup(Wi[k], q);
        }
        PrimeInfo &pi = c->h_pinfo[m];
        pi.q = q;
        int s = 64 - __builtin_clzll(q);
        pi.br.q = q;
        pi.br.sh = s - 2;
        pi.br.mu = (u64)(((u128)1 << (62 + s)) / q);
        pi.ninv = h_invmod((u64)N, q);
        pi.ninvp = h_shoup(pi.ninv, q);
        pi.ninvw1 = h_mulmod(pi.ninv, Wi[1], q);
        pi.ninvw1p = h_shoup(pi.ninvw1, q);
        pi.p_mod = c->p % q;
        pi.p_modp = h_shoup(pi.p_mod, q);
        // fp64 constants: integers below 2^50 are exact doubles and the
        // quotients are correctly rounded
        pi.qd = (double)q;
        pi.qinv = 1.0 / pi.qd;
        pi.ninv_d = (double)pi.ninv;
        pi.ninv_q = pi.ninv_d / pi.qd;
        pi.ninvw1_d = (double)pi.ninvw1;
        pi.ninvw1_q = pi.ninvw1_d / pi.qd;
        set_fpair(pi.p_f, c->p, q);
        set_fpair(pi.two25_f, (u64)1 << 25, q);
        for (int k = 1; k <= 3; k++) {
            pi.w123[k - 1][0] = W[k];
            pi.w123[k - 1][1] = Wp[k];
            set_fpair(pi.w123_f[k - 1], W[k], q);
        }
        for (int k = 2; k <= 3; k++) {
            pi.wi23[k - 2][0] = Wi[k];
            pi.wi23[k - 2][1] = Wip[k];
            set_fpair(pi.wi23_f[k - 2], Wi[k], q);
        }
    }
    c->tw = upload(tw.data(), tw.size());
    if (*std::max_element(c->mod.begin(), c->mod.end()) < ((u64)1 << 50)) {
        std::vector<double> twf(tw.size());
        for (int m = 0; m < nm; m++) {
            const u64 *W = &tw[(size_t)m * 4 * N], *Wi = W + 2 * N;
            double *F = &twf[(size_t)m * 4 * N], qd = (double)c->mod[m];
            for (int k = 0; k < N; k++) {
                F[k] = (double)W[k];
                F[2 * N + k] = (double)Wi[k];
                // W[2^k] and Winv[2^k], k < 4, are the transforms' multipliers
                // for derived twiddles: held centred (|w| <= q/2), which keeps
                // the derived twiddles below 5q/8 (any butterfly takes either form)
                if (k == 1 || k == 2 || k == 4 || k == 8) {
                    if (F[k] > 0.5 * qd) F[k] -= qd;
                    if (F[2 * N + k] > 0.5 * qd) F[2 * N + k] -= qd;
                }
                F[N + k] = F[k] / qd;
                F[3 * N + k] = F[2 * N + k] / qd;
            }
        }
        c->twf = upload(twf.data(), twf.size());
    }
    c->pinfo = upload(c->h_pinfo.data(), nm);

    // base-conversion and modulus-switching plans (fp64 twins when every
    // prime is below 2^50)
    {
        auto md = std::make_unique<ModDownPlan>();
        std::vector<ModSwitchPlan> ms;
        build_plans(c, set_shoup, c->h_modup, *md, ms);
        c->modup = upload(c->h_modup.data(), c->h_modup.size());
        c->moddown = upload(md.get(), 1);
        c->modsw = upload(ms.data(), nQ);
        if (c->twf) {
            std::vector<ModUpPlan> mu;
            build_plans(c, set_fpair, mu, *md, ms);
            c->modup_f = upload(mu.data(), mu.size());
            c->moddown_f = upload(md.get(), 1);
            c->modsw_f = upload(ms.data(), nQ);
            build_modup_mfma(c);
        }
    }

    // decryption: Garner tables
    auto g = std::make_unique<GarnerTable>();
    std::memset(g.get(), 0, sizeof(GarnerTable));
    u64 run = 1 % c->p;
    for (int i = 0; i < nQ; i++) {
        u64 q = c->mod[i];
        for (int j = 0; j < i; j++) set_shoup(g->inv[i][j], h_invmod(c->mod[j] % q, q), q);
        g->one_p[i] = (u64)(((u128)1 << 64) / q);
        g->mprod_p[i] = run;
        run = h_mulmod(run, q % c->p, c->p);
        g->qprod_p[i] = run;
    }
    c->garner = upload(g.get(), 1);
    const std::vector<u64> zeros((size_t)c->N, 0);
    c->zeros = upload(zeros.data(), zeros.size());
}

}  // namespace bc

namespace {
// frees a device table (no runtime call for one never allocated)
template <class T>
void dfree(T *p) {
    if (p) (void)hipFree((void *)p);
}
}  // namespace

bc_ctx::~bc_ctx() {
    if (biv_tab) (void)hipFree(biv_tab);
    graphs.reset();
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
    for (auto s : split_streams) (void)hipStreamDestroy(s);
    for (auto e : split_done) (void)hipEventDestroy(e);
    if (split_fork) (void)hipEventDestroy(split_fork);
    dfree(tw);
    dfree(twf);
    dfree(pinfo);
    dfree(modup);
    dfree(moddown);
    dfree(modsw);
    dfree(modup_f);
    dfree(moddown_f);
    dfree(modsw_f);
    for (auto &T : modup_mfma) {
        dfree(T.w8);
        dfree(T.corr);
    }
    dfree(garner);
    dfree(zeros);
    for (auto &kv : ps_coef) dfree(kv.second);
}

bc_keys::~bc_keys() {
    dfree(s_ntt);
    dfree(pk);
    dfree(rlk);
    for (auto p : gk) dfree(p);
    for (auto p : perm) dfree(p);
}
