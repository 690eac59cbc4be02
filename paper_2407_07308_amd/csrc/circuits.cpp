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
    V add_const(const V &a, int64_t v) {
        V o = alloc_ct(c, a.count, a.level, a.ncomp);
        each(o, a, nullptr, [&](const V &oo, const V &x, const V &) { bc::add_const(c, x, v, oo, st); });
        return o;
    }
    int level(const V &a) { return a.level; }
    V slice(const V &a, int first, int n) { return a.slice(first, n, c->N); }
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

}  // namespace

// ---------------------------------------------------------------- entry points

CompareResult compare(bc_ctx *c, const bc_keys *k, int ndig, const CtB *A, const CtB *B, bool want_mm, hipStream_t st) {
    BC_REQUIRE(ndig >= 1 && ndig <= 16, BC_ERR_ARG, "ndigits must be in [1, 16]");
    const int G = A[0].count, L0 = A[0].level;
    for (int d = 0; d < ndig; d++) {
        BC_REQUIRE(A[d].count == G && B[d].count == G, BC_ERR_ARG, "every plane needs the same count");
        BC_REQUIRE(A[d].level == L0 && B[d].level == L0, BC_ERR_ARG, "every plane needs the same level");
        BC_REQUIRE(A[d].ncomp == 2 && B[d].ncomp == 2, BC_ERR_ARG, "planes must have 2 components");
    }
    Shape sh = ps_shape(c->p);
    if (c->lt_c.empty()) {
        std::lock_guard<std::mutex> g(c->table_mu);
        if (c->lt_c.empty()) c->lt_c = lt_coefficients(c->p);
    }
    DevEval ev{c, k, st, c->exec_mode == BC_EXEC_PER_OP};
    const int N = c->N;
    // the planes of every group as one batch, plane-major, read straight from
    // the caller's planes: Z = A - B at the input level
    CtB Z = alloc_ct(c, ndig * G, L0, 2);
    for (int d = 0; d < ndig; d++)
        ev.each(Z.slice(d * G, G, N), A[d], &B[d],
                [&](const CtB &oo, const CtB &x, const CtB &y) { bc::add_sub(c, x, y, oo, true, st); });
    auto fz = lt_poly(ev, Z, sh, ndig * G, c->lt_c[c->p - 1]);
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

void compare_levels(const NoiseModel &m, int in_level, double in_noise, int ndig, bool want_mm, CircuitNoise *out) {
    Shape sh = ps_shape((u64)m.p);
    NoiseEval ev{&m};
    NoiseEval::V in{in_level, in_noise};
    m.require(in_level, in_noise, "comparison input");
    auto fz = lt_poly(ev, ev.sub(in, in), sh, 1, (int64_t)(m.p - 1) / 2);
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
