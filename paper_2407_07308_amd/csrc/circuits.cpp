// circuits.cpp -- the univariate less-than circuit, lexicographic combination,
// max / min, on batches of digit planes.
//
// Paper, Introduction: the univariate circuit computes LT(X, Y) = f(X - Y)
// with about sqrt(p-3) + O(log p) non-scalar multiplications.  Paper,
// Background, "Word-wise Universal FHE Scheme": integers are split into F_p
// digits, LT and EQ are evaluated per digit and combined in lexicographic
// order.  f is the degree p-1 interpolant of the indicator of
// [(p+1)/2, p-1] (x - y "negative"); it is exact as [x < y] for digits in
// [0, (p-1)/2].
//
// Batching: every plane of every group is one ciphertext of a single batch,
// so each step of the schedule is one launch sequence for the whole batch;
// the Paterson-Stockmeyer blocks are laid out in bit-reversed block order so
// that every round of the block tree is one batched multiplication.
//
// Every "x + y z" of the schedule (a node of the block tree, a lexicographic
// step, max and min) is one multiply-accumulate: x is added to the tensor of
// y and z before relinearisation and the modulus switch, so the sum is
// switched once (x is never below the product's level here).

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "ops.h"

namespace bc {

namespace {

// c_k = -sum_{z in [(p+1)/2, p-1]} z^(-k) mod p (k = 1 .. p-1), c_0 = 0: the
// inverse transform over F_p^* of the indicator (sum_z z^(j-k) = -[j = k mod p-1]).
std::vector<int64_t> lt_coefficients(u64 p) {
    std::vector<int64_t> c(p, 0);
    for (u64 k = 1; k <= p - 1; k++) {
        u64 s = 0;
        for (u64 z = (p + 1) / 2; z <= p - 1; z++) s = (s + h_powmod(h_invmod(z, p), k, p)) % p;
        c[k] = (int64_t)((p - s) % p);
    }
    return c;
}

struct Shape {
    int e, b, nblk;
    std::vector<int> odd;
};

Shape ps_shape(u64 p) {
    u64 pm1 = p - 1;
    BC_REQUIRE((pm1 & (pm1 - 1)) == 0, BC_ERR_PARAM, "the comparison schedule needs p - 1 a power of two");
    Shape s;
    s.e = __builtin_ctzll(pm1);
    s.b = 1 << ((s.e + 1) / 2);
    s.nblk = (int)(pm1 / s.b);
    for (int k = 1; k < s.b; k += 2) s.odd.push_back(k);
    return s;
}

// ---------------------------------------------------------------- evaluators

// Levels and noise estimates of the schedule, evaluated on the host before
// any launch: every step is checked against the budget of its level
// (BC_ERR_LEVEL when the circuit does not fit the chain).
struct NoiseEval {
    struct V {
        int lv = 0;
        double nb = 0;
    };
    const NoiseModel *m;
    int count = 1;
    V mul(V a, V b) { return mul_add(a, b, V{std::max(a.lv, b.lv), -INFINITY}); }
    V mul_add(V a, V b, V c) {
        const int lv = std::min(a.lv, b.lv);  // the addend is never below the product
        V o{lv > 0 ? lv - 1 : 0, m->product(lv, a.nb, b.nb, c.nb)};
        m->require(lv, o.nb, "comparison circuit");
        if (lv > 0) o.nb = m->mod_switch(lv, o.nb);
        m->require(o.lv, o.nb, "comparison circuit");
        return o;
    }
    V add(V a, V b) {
        V o{std::min(a.lv, b.lv), m->add(a.nb, b.nb)};
        m->require(o.lv, o.nb, "comparison circuit");
        return o;
    }
    V sub(V a, V b) { return add(a, b); }
    V rotate(V a, int) {
        V o{a.lv, m->rotate(a.lv, a.nb)};
        m->require(o.lv, o.nb, "comparison circuit");
        return o;
    }
    V mul_scalar(V a, int64_t c) { return V{a.lv, m->scalar(a.nb, (double)std::llabs(c))}; }
    V add_const(V a, int64_t) { return V{a.lv, m->add_const(a.nb)}; }
    int level(V a) { return a.lv; }
    V to_level(V a, int lv) { return V{std::min(a.lv, lv), a.nb}; }
    // every block sums b/2 babies with centred coefficients below p/2
    V blocks(const std::vector<V> &babies, int lv, int b, int) {
        double nb = -INFINITY;
        for (const V &x : babies) nb = std::max(nb, x.nb);
        V o{lv, m->scalar(nb, (double)(b / 2) * (m->p - 1) / 2)};
        m->require(lv, o.nb, "comparison circuit");
        return o;
    }
    V slice(V a, int, int) { return a; }
    // the batches pw[idx[j]] brought to level lv, as one batch
    V gather(const std::vector<V> &pw, const std::vector<int> &idx, int lv) {
        V o{lv, -INFINITY};
        for (int j : idx) o.nb = std::max(o.nb, pw[j].nb);
        return o;
    }
    // sums of in's blocks with integer weights (see BivNoise)
    template <class Tab>
    V lincomb_wide(const V &in, const Tab &t, bool final) {
        V o{in.lv, m->scalar(in.nb, final ? t.sum_abs : t.g_abs)};
        if (!final) o.nb = m->add_const(o.nb);
        m->require(o.lv, o.nb, "comparison circuit");
        return o;
    }
};

struct DevEval {
    typedef CtB V;
    bc_ctx *c;
    const bc_keys *k;
    hipStream_t st;
    bool per_op = false;  // one ciphertext per launch (the unbatched reference path)

    // Applies f(out_slice, a_slice, b_slice) per ciphertext when per_op is set.
    template <class F>
    void each(const V &out, const V &a, const V *b, F &&f) {
        if (!per_op) {
            f(out, a, b ? *b : a);
            return;
        }
        const int N = c->N;
        for (int i = 0; i < a.count; i++)
            f(out.slice(i, 1, N), a.slice(i, 1, N), b ? b->slice(i % b->count, 1, N) : a.slice(i, 1, N));
    }
    V mul(const V &a, const V &b) {
        V o = alloc_ct(c, a.count, out_level_mul(a.level, b.level), 2);
        each(o, a, &b, [&](const V &oo, const V &x, const V &y) { bc::mul_relin(c, k, x, y, oo, st); });
        return o;
    }
    // a b + d: the sum is formed before the product's relinearisation and
    // modulus switch (one switch instead of one for the product and one for d)
    V mul_add(const V &a, const V &b, const V &d) {
        V o = alloc_ct(c, a.count, out_level_mul(a.level, b.level), 2);
        if (!per_op) {
            bc::mul_relin_add(c, k, a, b, d, o, st);
            return o;
        }
        const int N = c->N;
        for (int i = 0; i < a.count; i++)
            bc::mul_relin_add(c, k, a.slice(i, 1, N), b.slice(i % b.count, 1, N), d.slice(i, 1, N), o.slice(i, 1, N), st);
        return o;
    }
    V add(const V &a, const V &b) {
        V o = alloc_ct(c, a.count, std::min(a.level, b.level), a.ncomp);
        each(o, a, &b, [&](const V &oo, const V &x, const V &y) { bc::add_sub(c, x, y, oo, false, st); });
        return o;
    }
    V sub(const V &a, const V &b) {
        V o = alloc_ct(c, a.count, std::min(a.level, b.level), a.ncomp);
        each(o, a, &b, [&](const V &oo, const V &x, const V &y) { bc::add_sub(c, x, y, oo, true, st); });
        return o;
    }
    V mul_scalar(const V &a, int64_t v) {
        V o = alloc_ct(c, a.count, a.level, a.ncomp);
        each(o, a, nullptr, [&](const V &oo, const V &x, const V &) { bc::mul_scalar(c, x, v, oo, st); });
        return o;
    }
    V rotate(const V &a, int steps) {
        V o = alloc_ct(c, a.count, a.level, 2);
        each(o, a, nullptr, [&](const V &oo, const V &x, const V &) { bc::rotate(c, k, x, steps, oo, st); });
        return o;
    }
    V add_const(const V &a, int64_t v) {
        V o = alloc_ct(c, a.count, a.level, a.ncomp);
        each(o, a, nullptr, [&](const V &oo, const V &x, const V &) { bc::add_const(c, x, v, oo, st); });
        return o;
    }
    int level(const V &a) { return a.level; }
    V slice(const V &a, int first, int n) { return a.slice(first, n, c->N); }
    V to_level(const V &a, int lv) {
        V o = alloc_ct(c, a.count, lv, a.ncomp);
        bc::to_level_into(c, a, o, st);
        return o;
    }
    V gather(const std::vector<V> &pw, const std::vector<int> &idx, int lv) {
        const int cnt = pw[idx[0]].count;
        V o = alloc_ct(c, (int)idx.size() * cnt, lv, 2);
        for (size_t j = 0; j < idx.size(); j++) bc::to_level_into(c, pw[idx[j]], o.slice((int)j * cnt, cnt, c->N), st);
        return o;
    }
    // the g_k(S) of the bivariate circuit from the gathered S powers, or
    // (final) LT from the gathered T_k and Z^(p-1) (see BivTable)
    template <class Tab>
    V lincomb_wide(const V &in, const Tab &t, bool final) {
        const int M = final ? t.K + 1 : t.M, K = final ? 1 : t.K;
        const int cnt = in.count / M;
        V o = alloc_ct(c, K * cnt, in.level, 2);
        if (!final && t.W8)
            launch_lincomb_wide_mfma(c, in.data, o.data, t.W8, t.c0, t.corr, M, K, cnt, in.level + 1, st);
        else
            launch_lincomb_wide(c, in.data, o.data, final ? t.Wsum : t.W, final ? t.c0sum : t.c0, M, K, cnt,
                                in.level + 1, st);
        BC_HIP(hipGetLastError());
        return o;
    }
    // blocks B_t = sum_{k odd < b} c_{tb+k} Z^k for every t at level lv (each
    // baby's lowest lv + 1 limbs: alignment by dropping primes), stored at
    // bit-reversed t
    V blocks(const std::vector<V> &babies, int lv, int b, int nblk);
};

// Linear-combination coefficients of the Paterson-Stockmeyer blocks, centred
// in (-p/2, p/2].  With fp64 arithmetic (and p small enough, see k_lincomb)
// they are one table of doubles [nblk][nbaby], the same for every prime;
// otherwise Shoup pairs [nblk][nbaby][nl][2] of their residues mod q_i.
const u64 *ps_coef_table(bc_ctx *c, int level, int b, int nblk) {
    std::lock_guard<std::mutex> g(c->table_mu);
    const bool small = lincomb_small(c);
    const int key = small ? -1 : level;
    auto it = c->ps_coef.find(key);
    if (it != c->ps_coef.end()) return it->second;
    if (c->lt_c.empty()) c->lt_c = lt_coefficients(c->p);
    const int nbaby = b / 2, nl = level + 1;
    std::vector<u64> tab;
    if (small) {
        tab.resize((size_t)nblk * nbaby);
        for (int t = 0; t < nblk; t++)
            for (int kk = 0; kk < nbaby; kk++) {
                const double cv = (double)centred(c, c->lt_c[(size_t)t * b + 2 * kk + 1]);
                std::memcpy(&tab[(size_t)t * nbaby + kk], &cv, sizeof(double));
            }
    } else {
        tab.resize((size_t)nblk * nbaby * nl * 2);
        for (int t = 0; t < nblk; t++)
            for (int kk = 0; kk < nbaby; kk++) {
                int64_t cv = centred(c, c->lt_c[(size_t)t * b + 2 * kk + 1]);
                for (int i = 0; i < nl; i++) {
                    u64 q = c->mod[i];
                    u64 r = cv >= 0 ? (u64)cv % q : q - (u64)(-cv) % q;
                    u64 *w = &tab[(((size_t)t * nbaby + kk) * nl + i) * 2];
                    w[0] = r % q;
                    w[1] = h_shoup(w[0], q);
                }
            }
    }
    u64 *d = nullptr;
    BC_HIP(hipMalloc(&d, sizeof(u64) * tab.size()));
    BC_HIP(hipMemcpy(d, tab.data(), sizeof(u64) * tab.size(), hipMemcpyHostToDevice));
    c->ps_coef[key] = d;
    return d;
}

DevEval::V DevEval::blocks(const std::vector<V> &babies, int lv, int b, int nblk) {
    const int count = babies[0].count, nbaby = (int)babies.size();
    const u64 *coef = ps_coef_table(c, lv, b, nblk);
    V out = alloc_ct(c, nblk * count, lv, 2);
    std::vector<const u64 *> bp;
    std::vector<int> nlb;
    for (auto &x : babies) {
        bp.push_back(x.data);
        nlb.push_back(x.level + 1);
    }
    int bits = __builtin_ctz(nblk);
    std::vector<int> pos(nblk);
    for (int t = 0; t < nblk; t++) pos[t] = bit_reverse(t, bits);
    if (!per_op) {
        launch_lincomb(c, bp.data(), nlb.data(), pos.data(), coef, out.data, nbaby, nblk, count, 0, count, lv + 1, st);
    } else {
        for (int i = 0; i < count; i++) {
            std::vector<const u64 *> bi;
            for (auto &x : babies) bi.push_back(x.data + (size_t)i * x.ct_words(c->N));
            launch_lincomb(c, bi.data(), nlb.data(), pos.data(), coef, out.data, nbaby, nblk, count, i, 1, lv + 1, st);
        }
    }
    BC_HIP(hipGetLastError());
    return out;
}

// f(Z) and Z^(p-1) by the Paterson-Stockmeyer schedule described above.
template <class Ev>
std::pair<typename Ev::V, typename Ev::V> lt_poly(Ev &ev, const typename Ev::V &Z, const Shape &sh, int count,
                                                  int64_t ctop) {
    typedef typename Ev::V V;
    const int b = sh.b;
    std::vector<V> pw(b + 1);
    std::vector<bool> have(b + 1, false);
    pw[1] = Z;
    have[1] = true;
    for (int a = 1; 2 * a <= b / 2; a *= 2) {
        pw[2 * a] = ev.mul(pw[a], pw[a]);
        have[2 * a] = true;
    }
    for (int k = 3; k < b; k += 2) {
        int hi = 1 << (31 - __builtin_clz(k));
        pw[k] = ev.mul(pw[hi], pw[k - hi]);
        have[k] = true;
    }
    std::vector<V> giants;
    giants.push_back(b >= 2 ? ev.mul(pw[b / 2], pw[b / 2]) : Z);
    while (((int64_t)b << giants.size()) <= (int64_t)(sh.nblk * b)) giants.push_back(ev.mul(giants.back(), giants.back()));
    int lv = ev.level(pw[1]);
    for (int k : sh.odd) lv = std::min(lv, ev.level(pw[k]));
    std::vector<V> babies;  // brought to lv by the blocks step (lowest lv + 1 limbs)
    for (int k : sh.odd) babies.push_back(pw[k]);
    V H = ev.blocks(babies, lv, b, sh.nblk);
    int len = sh.nblk, r = 0;
    while (len > 1) {
        int half = len / 2;
        V lo = ev.slice(H, 0, half * count), hi = ev.slice(H, half * count, half * count);
        H = ev.mul_add(hi, giants[r], lo);
        len = half;
        r++;
    }
    V f = ev.add(H, ev.mul_scalar(giants.back(), ctop));
    return {f, giants.back()};
}

// LT over planes (plane-major batches of `count` groups), EQ_d = 1 - Z_d^(p-1),
// LT = LT_0 + EQ_0 (LT_1 + EQ_1 (... LT_{n-1})).
template <class Ev>
typename Ev::V lexicographic(Ev &ev, const typename Ev::V &f, const typename Ev::V &top, int ndig, int count) {
    typedef typename Ev::V V;
    V eq = ev.add_const(ev.mul_scalar(top, -1), 1);
    V acc = ev.slice(f, (ndig - 1) * count, count);
    for (int d = ndig - 2; d >= 0; d--)
        acc = ev.mul_add(ev.slice(eq, d * count, count), acc, ev.slice(f, d * count, count));
    return acc;
}

// ------------------------------------------------------- bivariate circuit
// (Introduction: the bivariate circuit, exact for every pair of digits; the
// paper prints no polynomial or schedule)

// c[m p + k]: coefficient of S^m Z^k in the interpolant G(S, Z) of [x < y]
// over F_p^2 with S = x + y, Z = x - y (p odd).  Interpolation one axis at a
// time: the interpolant of h over F_p has a_0 = h(0) and, for j >= 1,
// a_j = -sum_{t != 0} h(t) t^-j - [j = p - 1] h(0) (from the indicator
// 1 - (x - t)^(p-1) of each point).
std::vector<int64_t> bivariate_coefficients(u64 p) {
    const size_t P = (size_t)p;
    std::vector<u64> tinv(P * P);  // tinv[t p + j] = t^-j
    for (u64 t = 1; t < p; t++) {
        const u64 ti = h_invmod(t, p);
        u64 v = 1;
        for (u64 j = 0; j < p; j++) {
            tinv[t * P + j] = v;
            v = v * ti % p;
        }
    }
    auto interp = [&](const std::vector<u64> &h, std::vector<u64> &a) {
        a.assign(P, 0);
        a[0] = h[0];
        for (u64 j = 1; j < p; j++) {
            u64 acc = 0;
            for (u64 t = 1; t < p; t++) acc = (acc + h[t] * tinv[t * P + j]) % p;
            if (j == p - 1) acc = (acc + h[0]) % p;
            a[j] = (p - acc) % p;
        }
    };
    const u64 inv2 = (p + 1) / 2;
    std::vector<u64> A1(P * P), h(P), a;
    for (u64 sv = 0; sv < p; sv++) {  // along z for each s
        for (u64 zv = 0; zv < p; zv++) {
            const u64 x = (sv + zv) % p * inv2 % p, y = (sv + p - zv) % p * inv2 % p;
            h[zv] = x < y ? 1 : 0;
        }
        interp(h, a);
        for (u64 k = 0; k < p; k++) A1[sv * P + k] = a[k];
    }
    std::vector<int64_t> c(P * P);
    for (u64 k = 0; k < p; k++) {  // then along s for each power of z
        for (u64 sv = 0; sv < p; sv++) h[sv] = A1[sv * P + k];
        interp(h, a);
        for (u64 m = 0; m < p; m++) c[m * P + k] = (int64_t)a[m];
    }
    return c;
}

// Weights of the bivariate circuit as the wide-combination kernel takes them
// (centred doubles): rows k' < K = (p-1)/2 of g_{2k'+1}(S) = sum_{m=1}^{p-1}
// c[m][2k'+1] S^m (+ c[0][2k'+1]), then one row for the final sum
// LT = sum_k T_k + (p+1)/2 Z^(p-1) (weights 1 ... 1, (p+1)/2; no constant).
struct BivTable {
    int K, M;
    const double *W, *c0, *Wsum, *c0sum;
    const int8_t *W8;  // the g_k weights as int8 [128][256] for the matrix cores (null: p too large)
    const int *corr;   // their weights equal to 128, listed per row
};
// What the noise estimate needs of the same weights: the largest total
// weight magnitude of one g_k (a bound, (p-1)/2 per weight) and of the sum.
struct BivNoise {
    int K, M;
    double g_abs, sum_abs;
};
BivNoise bivariate_noise(u64 p) {
    const int K = (int)(p - 1) / 2, M = (int)p - 1;
    return BivNoise{K, M, (double)M * (double)(p - 1) / 2 + 1, (double)K + (double)(p - 1) / 2};
}

BivTable bivariate_table(bc_ctx *c) {
    std::lock_guard<std::mutex> g(c->table_mu);
    const u64 p = c->p;
    const int K = (int)(p - 1) / 2, M = (int)p - 1;
    const int KP = (K + lincomb_wide_tile(K) - 1) / lincomb_wide_tile(K) * lincomb_wide_tile(K);
    const size_t nW = (size_t)KP * M, nS = (size_t)K + 1;
    if (!c->biv_tab) {
        BC_REQUIRE(p >= 3 && p < 512 && ((p - 1) & (p - 2)) == 0, BC_ERR_PARAM,
                   "the bivariate circuit needs p - 1 a power of two and p < 512");
        const std::vector<int64_t> cf = bivariate_coefficients(p);
        const size_t P = (size_t)p;
        // the schedule relies on the part even in Z being (p+1)/2 Z^(p-1)
        for (size_t k = 0; k < P; k += 2)
            for (size_t m = 0; m < P; m++)
                BC_REQUIRE(cf[m * P + k] == ((m == 0 && k == P - 1) ? (int64_t)(p + 1) / 2 : 0), BC_ERR_PARAM,
                           "bivariate interpolant: unexpected even part");
        auto cen = [&](int64_t v) { return (double)(v > (int64_t)(p - 1) / 2 ? v - (int64_t)p : v); };
        std::vector<double> host(nW + KP + nS + 1, 0.0);
        for (int kk = 0; kk < K; kk++)
            for (int mm = 0; mm < M; mm++) host[(size_t)kk * M + mm] = cen(cf[(size_t)(mm + 1) * P + 2 * kk + 1]);
        for (int kk = 0; kk < K; kk++) host[nW + kk] = cen(cf[2 * kk + 1]);
        for (int kk = 0; kk < K; kk++) host[nW + KP + kk] = 1.0;
        host[nW + KP + K] = cen((int64_t)(p + 1) / 2);
        // the matrix-core copy: int8 weights (128 is not one: listed apart)
        std::vector<int8_t> w8((size_t)kWideMfmaK * kWideMfmaM, 0);
        std::vector<int> corr(K + 1, 0), cm;
        if (K <= kWideMfmaK && M <= kWideMfmaM) {
            for (int kk = 0; kk < K; kk++) {
                for (int mm = 0; mm < M; mm++) {
                    const double v = host[(size_t)kk * M + mm];
                    if (v == 128.0) cm.push_back(mm);
                    else w8[(size_t)kk * kWideMfmaM + mm] = (int8_t)v;
                }
                corr[kk + 1] = (int)cm.size();
            }
        }
        corr.insert(corr.end(), cm.begin(), cm.end());
        // the int8 rows start on a 256-byte boundary (16-byte operand loads)
        const size_t bytes_d = (sizeof(double) * host.size() + 255) / 256 * 256;
        const size_t bytes = bytes_d + w8.size() + sizeof(int) * corr.size();
        char *d = nullptr;
        BC_HIP(hipMalloc(&d, bytes));
        BC_HIP(hipMemcpy(d, host.data(), sizeof(double) * host.size(), hipMemcpyHostToDevice));
        BC_HIP(hipMemcpy(d + bytes_d, w8.data(), w8.size(), hipMemcpyHostToDevice));
        BC_HIP(hipMemcpy(d + bytes_d + w8.size(), corr.data(), sizeof(int) * corr.size(), hipMemcpyHostToDevice));
        c->biv_tab = (double *)d;
        c->biv_mfma = K <= kWideMfmaK && M <= kWideMfmaM;
        c->biv_K = K;
        c->biv_M = M;
    }
    const double *d = c->biv_tab;
    const char *b = (const char *)d + (sizeof(double) * (nW + KP + nS + 1) + 255) / 256 * 256;
    return BivTable{K, M, d, d + nW, d + nW + KP, d + nW + KP + nS,
                    c->biv_mfma && c->mfma ? (const int8_t *)b : nullptr,
                    (const int *)(b + (size_t)kWideMfmaK * kWideMfmaM)};
}

// The bivariate interpolant of [x < y] on Z = X - Y, S = X + Y (batches of
// `count` ciphertexts), p - 1 = 2^e:
//   LT = (p+1)/2 Z^(p-1) + sum_{k odd} Z^k g_k(S)
// (the part even in Z of the interpolant is (p+1)/2 Z^(p-1), since
// LT(x, y) + LT(y, x) = (x - y)^(p-1)).  Power ladders: X^(2^a) by squaring,
// X^(2^a + r) = X^(2^a) X^r for r < 2^a (every r for S, odd r for Z), each
// block of a ladder one batched product against the broadcast X^(2^a); the
// S powers gathered at the level of S^(p-1) and combined into all g_k by one
// wide linear combination; the odd Z powers gathered at the same level; one
// batched product T_k = Z^k g_k; LT by one more wide combination of the T_k
// and (p+1)/2 Z^(p-1).  Returns (LT, Z^(p-1)).
template <class Ev, class Tab>
std::pair<typename Ev::V, typename Ev::V> lt_bivariate(Ev &ev, const typename Ev::V &Z, const typename Ev::V &S,
                                                       int count, int P1, const Tab &tab) {
    typedef typename Ev::V V;
    auto ladder = [&](const V &B, bool odd_only) {
        std::vector<V> pw(P1 + 1);
        pw[1] = B;
        for (int a = 1; a < P1; a *= 2) pw[2 * a] = ev.mul(pw[a], pw[a]);
        for (int a = 2; a < P1; a *= 2) {
            std::vector<int> rs;
            for (int r = 1; r < a; r++)
                if (!odd_only || (r & 1)) rs.push_back(r);
            const V prod = ev.mul(ev.gather(pw, rs, ev.level(pw[a])), pw[a]);
            for (size_t j = 0; j < rs.size(); j++) pw[a + rs[j]] = ev.slice(prod, (int)j * count, count);
        }
        return pw;
    };
    V G;
    int lv;
    {
        std::vector<V> sp = ladder(S, false);
        lv = ev.level(sp[P1]);
        std::vector<int> ms;
        for (int m = 1; m <= P1; m++) ms.push_back(m);
        const V SC = ev.gather(sp, ms, lv);
        sp.clear();  // only the gathered copies are read from here on
        G = ev.lincomb_wide(SC, tab, false);
    }
    std::vector<V> zp = ladder(Z, true);
    std::vector<int> ks;
    for (int k = 1; k < P1; k += 2) ks.push_back(k);
    const V T = ev.mul(ev.gather(zp, ks, lv), G);
    G = V();
    const V top = zp[P1];
    zp.clear();
    // the T_k and Z^(p-1) as one batch of K + 1 blocks at T's level
    std::vector<V> parts;
    for (size_t k = 0; k < ks.size(); k++) parts.push_back(ev.slice(T, (int)k * count, count));
    parts.push_back(top);
    std::vector<int> all;
    for (size_t k = 0; k < parts.size(); k++) all.push_back((int)k);
    const V LT = ev.lincomb_wide(ev.gather(parts, all, ev.level(T)), tab, true);
    return {LT, top};
}

// ------------------------------------------------------- slot-packed digits
// (Background, "Word-wise Universal FHE Scheme": the digits' LT and EQ
// combined by ShiftMul -- shift the ciphertext, multiply by the equality
// result -- and ShiftAdd -- a summation done by shifting)

// Per-slot (LT, Z^(p-1)) of the digit batches X, Y (`count` ciphertexts
// each) by the chosen digit circuit.
template <class Ev, class BT>
std::pair<typename Ev::V, typename Ev::V> digit_circuit(Ev &ev, const typename Ev::V &X, const typename Ev::V &Y,
                                                        int count, int circuit, u64 p, const BT &biv, int64_t ctop) {
    const typename Ev::V Z = ev.sub(X, Y);
    if (circuit == BC_CIRCUIT_BIVARIATE) return lt_bivariate(ev, Z, ev.add(X, Y), count, (int)p - 1, biv);
    return lt_poly(ev, Z, ps_shape(p), count, ctop);
}

// Integers packed l digits each into consecutive slots of a row (most
// significant first): from the per-slot L = LT and E = 1 - Z^(p-1), one round
// per shift s = 1, 2, ..., l/2 (rotation by s brings slot j + s of the row to
// slot j):
//   L <- L + E rot(L, s)   (one multiply-accumulate),   E <- E rot(E, s)
// (E not in the last round).  After the round with shift s, slot k l + i
// (i a multiple of 2s) holds the lexicographic (LT, EQ) of digits i .. i+2s-1
// of integer k: slot k l ends with integer k's LT.
template <class Ev>
typename Ev::V packed_tree(Ev &ev, typename Ev::V L, const typename Ev::V &top, int l) {
    typedef typename Ev::V V;
    V E = ev.add_const(ev.mul_scalar(top, -1), 1);
    for (int s = 1; s < l; s *= 2) {
        const bool last = 2 * s >= l;
        const V Lr = ev.rotate(L, s);
        V Er;
        if (!last) Er = ev.rotate(E, s);
        L = ev.mul_add(E, Lr, L);
        if (!last) E = ev.mul(E, Er);
    }
    return L;
}

// Minimum (maximum) over windows of `window` = 2^r slots of a row: round t
// (s = 2^t) compares X with Y = rot(X, s) slot by slot and keeps
// Y + L (X - Y) (min) or X + L (Y - X) (max), X and Y brought to L's level.
// Slot j ends with the min (max) of slots j .. j + window - 1 of its row
// (cyclically); windows at multiples of `window` are disjoint tournaments.
template <class Ev, class BT>
typename Ev::V tournament_rounds(Ev &ev, typename Ev::V X, int count, int window, bool want_max, int circuit, u64 p,
                                 const BT &biv, int64_t ctop) {
    typedef typename Ev::V V;
    for (int s = 1; s < window; s *= 2) {
        const V Y = ev.rotate(X, s);
        const V L = digit_circuit(ev, X, Y, count, circuit, p, biv, ctop).first;
        const int lv = ev.level(L);
        const V Xl = ev.to_level(X, lv), Yl = ev.to_level(Y, lv);
        X = want_max ? ev.mul_add(L, ev.sub(Yl, Xl), Xl) : ev.mul_add(L, ev.sub(Xl, Yl), Yl);
    }
    return X;
}

void check_packed_args(const bc_ctx *c, int circuit, int len, const char *what) {
    BC_REQUIRE(circuit == BC_CIRCUIT_UNIVARIATE || circuit == BC_CIRCUIT_BIVARIATE, BC_ERR_ARG, "unknown circuit");
    BC_REQUIRE(len >= 1 && (len & (len - 1)) == 0 && len <= c->M / 2, BC_ERR_ARG, what);
}

// The digit circuit's tables on the device side.
struct DevDigit {
    BivTable biv{};
    int64_t ctop = 0;
};
DevDigit dev_digit(bc_ctx *c, int circuit) {
    DevDigit d;
    if (circuit == BC_CIRCUIT_BIVARIATE) {
        d.biv = bivariate_table(c);
        BC_REQUIRE(use_fp64(c), BC_ERR_PARAM, "the bivariate circuit needs primes below 2^50");
    } else {
        (void)ps_shape(c->p);
        if (c->lt_c.empty()) {
            std::lock_guard<std::mutex> g(c->table_mu);
            if (c->lt_c.empty()) c->lt_c = lt_coefficients(c->p);
        }
        d.ctop = c->lt_c[c->p - 1];
    }
    return d;
}
BivNoise noise_biv(const NoiseModel &m, int circuit) {
    const u64 p = (u64)m.p;
    if (circuit == BC_CIRCUIT_BIVARIATE)
        BC_REQUIRE(p >= 3 && p < 512 && ((p - 1) & (p - 2)) == 0, BC_ERR_PARAM,
                   "the bivariate circuit needs p - 1 a power of two and p < 512");
    return bivariate_noise(p);
}

}  // namespace

// ---------------------------------------------------------------- entry points

CtB compare_packed(bc_ctx *c, const bc_keys *k, const CtB &A, const CtB &B, int l, int circuit, hipStream_t st) {
    check_packed_args(c, circuit, l, "digits per integer must be a power of two up to half the slots");
    BC_REQUIRE(A.count == B.count && A.level == B.level && A.ncomp == 2 && B.ncomp == 2, BC_ERR_ARG,
               "packed operands: same count and level, 2 components");
    DevEval ev{c, k, st, c->exec_mode == BC_EXEC_PER_OP};
    const DevDigit d = dev_digit(c, circuit);
    const auto fz = digit_circuit(ev, A, B, A.count, circuit, c->p, d.biv, d.ctop);
    return packed_tree(ev, fz.first, fz.second, l);
}

CtB tournament(bc_ctx *c, const bc_keys *k, const CtB &X, int window, bool want_max, int circuit, hipStream_t st) {
    check_packed_args(c, circuit, window, "the window must be a power of two up to half the slots");
    BC_REQUIRE(X.ncomp == 2, BC_ERR_ARG, "tournament input: 2 components");
    DevEval ev{c, k, st, c->exec_mode == BC_EXEC_PER_OP};
    const DevDigit d = dev_digit(c, circuit);
    return tournament_rounds(ev, X, X.count, window, want_max, circuit, c->p, d.biv, d.ctop);
}

// The mod-extract step (Background, "Word-wise Universal FHE Scheme"): digit
// k of a slot's F_{p^d} element is d^-1 Tr(x^-k m), the trace summing the d
// Frobenius images; it runs as log2(d) doublings z <- z + sigma(z), every
// digit and ciphertext of the batch in each launch.
void extract_digits(bc_ctx *c, const bc_keys *k, const CtB &in, const int *digits, int ndig, const CtB &out,
                    hipStream_t st) {
    const int N = c->N, d = N / c->M, nl = in.level + 1;
    BC_REQUIRE(in.ncomp == 2 && in.count >= 1, BC_ERR_ARG, "extraction input: 2 components");
    BC_REQUIRE(digits && ndig >= 1, BC_ERR_ARG, "no digits to extract");
    BC_REQUIRE(out.ncomp == 2 && out.level == in.level && out.count == in.count * ndig, BC_ERR_ARG,
               "extraction output: ndigits x count ciphertexts at the input's level");
    {
        const u64 *ib = in.data, *ie = ib + (size_t)in.count * in.ct_words(N);
        const u64 *ob = out.data, *oe = ob + (size_t)out.count * out.ct_words(N);
        BC_REQUIRE(oe <= ib || ie <= ob, BC_ERR_ARG, "extraction output overlaps its input");
    }
    for (int j = 0; j < ndig; j++)
        BC_REQUIRE(digits[j] >= 0 && digits[j] < d, BC_ERR_ARG, "digit index beyond the slot degree N/M");
    const std::vector<int> steps = frobenius_steps(c);
    for (int r : steps) {
        bool have = false;
        for (int i = 0; i < k->ngal; i++) have = have || k->steps[i] == r;
        BC_REQUIRE(have, BC_ERR_KEY, "no rotation key for a Frobenius step");
    }
    const size_t W = in.ct_words(N);
    for (int j = 0; j < ndig; j++)  // x^-k = x^(2N - k)
        launch_mul_monomial(c, in.data, out.data + (size_t)j * in.count * W, in.count, nl, 2,
                            (2 * N - digits[j]) % (2 * N), st);
    // z <- z + sigma(z) between out and tmp; the scalar d^-1 writes out
    CtB tmp = alloc_ct(c, out.count, out.level, 2);
    const CtB *z = &out, *zn = &tmp;
    for (int r : steps) {
        rotate_add(c, k, *z, r, *zn, st);
        std::swap(z, zn);
    }
    mul_scalar(c, *z, (int64_t)h_invmod((u64)(d % c->p), (u64)c->p), out, st);
}

void packed_levels(const NoiseModel &m, int in_level, double in_noise, int l, int circuit, int *lv, double *nb) {
    NoiseEval ev{&m};
    const NoiseEval::V in{in_level, in_noise};
    m.require(in_level, in_noise, "comparison input");
    const auto fz = digit_circuit(ev, in, in, 1, circuit, (u64)m.p, noise_biv(m, circuit), (int64_t)(m.p - 1) / 2);
    const NoiseEval::V L = packed_tree(ev, fz.first, fz.second, l);
    *lv = L.lv;
    *nb = L.nb;
}

void tournament_levels(const NoiseModel &m, int in_level, double in_noise, int window, int circuit, int *lv,
                       double *nb) {
    NoiseEval ev{&m};
    m.require(in_level, in_noise, "tournament input");
    const NoiseEval::V X = tournament_rounds(ev, NoiseEval::V{in_level, in_noise}, 1, window, false, circuit,
                                             (u64)m.p, noise_biv(m, circuit), (int64_t)(m.p - 1) / 2);
    *lv = X.lv;
    *nb = X.nb;
}

CompareResult compare(bc_ctx *c, const bc_keys *k, int ndig, const CtB *A, const CtB *B, bool want_mm, hipStream_t st,
                      int circuit) {
    BC_REQUIRE(circuit == BC_CIRCUIT_UNIVARIATE || circuit == BC_CIRCUIT_BIVARIATE, BC_ERR_ARG, "unknown circuit");
    BC_REQUIRE(ndig >= 1 && ndig <= 16, BC_ERR_ARG, "ndigits must be in [1, 16]");
    const int G = A[0].count, L0 = A[0].level;
    for (int d = 0; d < ndig; d++) {
        BC_REQUIRE(A[d].count == G && B[d].count == G, BC_ERR_ARG, "every plane needs the same count");
        BC_REQUIRE(A[d].level == L0 && B[d].level == L0, BC_ERR_ARG, "every plane needs the same level");
        BC_REQUIRE(A[d].ncomp == 2 && B[d].ncomp == 2, BC_ERR_ARG, "planes must have 2 components");
    }
    DevEval ev{c, k, st, c->exec_mode == BC_EXEC_PER_OP};
    const int N = c->N;
    // the planes of every group as one batch, plane-major, read straight from
    // the caller's planes: Z = A - B (and S = A + B) at the input level
    CtB Z = alloc_ct(c, ndig * G, L0, 2);
    for (int d = 0; d < ndig; d++)
        ev.each(Z.slice(d * G, G, N), A[d], &B[d],
                [&](const CtB &oo, const CtB &x, const CtB &y) { bc::add_sub(c, x, y, oo, true, st); });
    std::pair<CtB, CtB> fz;
    if (circuit == BC_CIRCUIT_BIVARIATE) {
        const BivTable tab = bivariate_table(c);
        BC_REQUIRE(use_fp64(c), BC_ERR_PARAM, "the bivariate circuit needs primes below 2^50");
        CtB S = alloc_ct(c, ndig * G, L0, 2);
        for (int d = 0; d < ndig; d++) bc::add_sub(c, A[d], B[d], S.slice(d * G, G, N), false, st);
        fz = lt_bivariate(ev, Z, S, ndig * G, (int)c->p - 1, tab);
    } else {
        Shape sh = ps_shape(c->p);
        if (c->lt_c.empty()) {
            std::lock_guard<std::mutex> g(c->table_mu);
            if (c->lt_c.empty()) c->lt_c = lt_coefficients(c->p);
        }
        fz = lt_poly(ev, Z, sh, ndig * G, c->lt_c[c->p - 1]);
    }
    Z = CtB();
    CompareResult r;
    r.lt = lexicographic(ev, fz.first, fz.second, ndig, G);
    if (want_mm) {
        // both operands at LT's level first: the differences are formed there
        auto at_lt = [&](const CtB *X) {
            CtB o = alloc_ct(c, ndig * G, r.lt.level, 2);
            for (int d = 0; d < ndig; d++)
                ev.each(o.slice(d * G, G, N), X[d], nullptr,
                        [&](const CtB &oo, const CtB &x, const CtB &) { bc::to_level_into(c, x, oo, st); });
            return o;
        };
        CtB Al = at_lt(A), Bl = at_lt(B);
        r.mx = ev.mul_add(ev.sub(Bl, Al), r.lt, Al);
        r.mn = ev.mul_add(ev.sub(Al, Bl), r.lt, Bl);
    }
    return r;
}

void compare_levels(const NoiseModel &m, int in_level, double in_noise, int ndig, bool want_mm, CircuitNoise *out,
                    int circuit) {
    BC_REQUIRE(circuit == BC_CIRCUIT_UNIVARIATE || circuit == BC_CIRCUIT_BIVARIATE, BC_ERR_ARG, "unknown circuit");
    NoiseEval ev{&m};
    NoiseEval::V in{in_level, in_noise};
    m.require(in_level, in_noise, "comparison input");
    std::pair<NoiseEval::V, NoiseEval::V> fz;
    if (circuit == BC_CIRCUIT_BIVARIATE) {
        const u64 p = (u64)m.p;
        BC_REQUIRE(p >= 3 && p < 512 && ((p - 1) & (p - 2)) == 0, BC_ERR_PARAM,
                   "the bivariate circuit needs p - 1 a power of two and p < 512");
        fz = lt_bivariate(ev, ev.sub(in, in), ev.add(in, in), 1, (int)p - 1, bivariate_noise(p));
    } else {
        fz = lt_poly(ev, ev.sub(in, in), ps_shape((u64)m.p), 1, (int64_t)(m.p - 1) / 2);
    }
    NoiseEval::V lt = lexicographic(ev, fz.first, fz.second, ndig, 1);
    out->lt_level = lt.lv;
    out->lt_noise = lt.nb;
    out->mm_level = lt.lv > 0 ? lt.lv - 1 : 0;
    out->mm_noise = 0;
    if (want_mm) {
        const NoiseEval::V al = ev.to_level(in, lt.lv);
        const NoiseEval::V mm = ev.mul_add(ev.sub(al, al), lt, al);
        out->mm_level = mm.lv;
        out->mm_noise = mm.nb;
    } else {
        // levels are reported either way
        out->mm_level = lt.lv > 0 ? lt.lv - 1 : 0;
    }
}

}  // namespace bc
