// ops.cpp -- BGV operations on batches of device ciphertexts.
//
// Ciphertexts stay in HBM in the NTT domain between operations; every
// operation is a short fixed sequence of batched kernel launches on one
// stream, each launch covering all ciphertexts, components and limbs of the
// batch (the whole residue matrix, as in the paper's "GPU-related
// Optimizations", instead of one launch per row or per ciphertext).
//
// Multiplication (tensor, then relinearisation by hybrid key switching, then
// one modulus switch) and rotation (automorphism, then key switching) are the
// operations the comparison circuit is made of (paper, Background, "Word-wise
// Universal FHE Scheme").

#include "ops.h"
#include "persist.h"

#include <algorithm>
#include <atomic>
#include <cstring>

namespace bc {

CtB alloc_ct(bc_ctx *c, int count, int level, int ncomp) {
    CtB x;
    x.count = count;
    x.level = level;
    x.ncomp = ncomp;
    x.own = make_buf(c, sizeof(u64) * (size_t)count * x.ct_words(c->N));
    x.data = (u64 *)x.own->p;
    return x;
}

CtB from_abi(const bc_ctx *c, const bc_ctb *x) {
    BC_REQUIRE(x && x->data, BC_ERR_ARG, "null ciphertext batch");
    BC_REQUIRE(x->count >= 1, BC_ERR_ARG, "empty ciphertext batch");
    BC_REQUIRE(x->level >= 0 && x->level < c->nQ, BC_ERR_LEVEL, "ciphertext level out of range");
    BC_REQUIRE(x->ncomp == 2 || x->ncomp == 3, BC_ERR_ARG, "ciphertexts have 2 or 3 components");
    CtB b;
    b.data = x->data;
    b.count = x->count;
    b.level = x->level;
    b.ncomp = x->ncomp;
    b.noise = c->noise.input(x->noise_bits);
    return b;
}

int64_t centred(const bc_ctx *c, int64_t v) {
    int64_t p = (int64_t)c->p;
    v %= p;
    if (v < 0) v += p;
    return v > (p - 1) / 2 ? v - p : v;
}

namespace {

// Transform jobs over a batch; split across launches when too many limbs.
struct Jobs {
    struct J {
        int off, prime, ioff;  // output limb slot, prime, input limb slot (out of place)
    };
    std::vector<J> l;
    void add(int off, int prime, int ioff = -1) { l.push_back({off, prime, ioff < 0 ? off : ioff}); }
};

// Transforms the jobs' limbs of `npoly` polys (stride `stride` words) in
// place, or, with `in`, reads limb ioff of poly j at in + j * in_stride and
// writes the result to the output slot.
void run_ntt(const bc_ctx *c, u64 *base, size_t stride, int npoly, const Jobs &j, bool inverse, hipStream_t st,
             const u64 *in = nullptr, size_t in_stride = 0) {
    for (size_t s = 0; s < j.l.size(); s += kMaxJobs) {
        LimbSet ls{};
        ls.base = base;
        ls.poly_stride = stride;
        ls.npoly = npoly;
        ls.nlimb = (int)std::min<size_t>(kMaxJobs, j.l.size() - s);
        ls.ibase = in;
        ls.ipoly_stride = in_stride;
        for (int k = 0; k < ls.nlimb; k++) {
            ls.off[k] = (int16_t)j.l[s + k].off;
            ls.prime[k] = (int16_t)j.l[s + k].prime;
            ls.ioff[k] = (int16_t)j.l[s + k].ioff;
        }
        if (inverse) ntt_inverse(c, ls, st);
        else ntt_forward(c, ls, st);
    }
}

// Part-limb transforms (ntt_parts_log(c) > 0), as run_ntt: forward, of limbs
// whose first stages their producer applied; inverse, leaving the last
// stages to the kernel that consumes the limbs.
// raw_in / raw_out: the limbs are read / written as reduced fp64 patterns
void run_ntt_parts(const bc_ctx *c, u64 *base, size_t stride, int npoly, const Jobs &j, bool inverse, hipStream_t st,
                   const u64 *in = nullptr, size_t in_stride = 0, bool raw_in = false, bool raw_out = false) {
    for (size_t s = 0; s < j.l.size(); s += kMaxJobs) {
        LimbSet ls{};
        ls.raw_in = raw_in;
        ls.raw_out = raw_out;
        ls.base = base;
        ls.poly_stride = stride;
        ls.npoly = npoly;
        ls.nlimb = (int)std::min<size_t>(kMaxJobs, j.l.size() - s);
        ls.ibase = in;
        ls.ipoly_stride = in_stride;
        for (int k = 0; k < ls.nlimb; k++) {
            ls.off[k] = (int16_t)j.l[s + k].off;
            ls.prime[k] = (int16_t)j.l[s + k].prime;
            ls.ioff[k] = (int16_t)j.l[s + k].ioff;
        }
        if (inverse) ntt_inverse_parts(c, ls, st);
        else ntt_forward_parts(c, ls, st);
    }
}

// Whether the key-switching kernels pass their intermediate limbs as reduced
// fp64 patterns: part-limb transforms with fp64 arithmetic, ordinary launches
// (the persistent executor's stages pass canonical words).
bool raw_handoff(const bc_ctx *c) { return c->raw_handoff && ntt_parts_log(c) > 0 && use_fp64(c) && !tl_rec; }

// all limbs of a [count][ncomp][nl][N] batch
Jobs all_limbs(int ncomp, int nl) {
    Jobs j;
    for (int k = 0; k < ncomp; k++)
        for (int i = 0; i < nl; i++) j.add(k * nl + i, i);
    return j;
}

void check_hip() { BC_HIP(hipGetLastError()); }

// Key switch of the NTT-domain polynomials X (stride x_stride per ciphertext,
// level `level`) with key [dnum][2][nmod][N]:
// out_c = base_c + ModDown(sum_j ModUp_j(X) * key_j,c), c = 0, 1.
// Digit decomposition, basis extension and inner product with the key:
// returns ACC[count][2][l+1+nP][N] = sum_j ModUp_j(X) * key_j,c (NTT domain).
BufP ks_accumulate(bc_ctx *c, const u64 *key, const u64 *X, size_t x_stride, int count, int level, hipStream_t st) {
    const int N = c->N, nl = level + 1, next = nl + c->nP, dnum = c->dnum;
    const int nact = level / c->alpha + 1;
    // MU[ct][j][e] holds digit j's new limbs; its own limbs are read from X
    BufP MU = make_buf(c, sizeof(u64) * (size_t)count * dnum * next * N);
    BufP XC = make_buf(c, sizeof(u64) * (size_t)count * nl * N);
    u64 *mu = (u64 *)MU->p, *xc = (u64 *)XC->p;
    Jobs jx;  // coefficient-domain copy of X
    for (int i = 0; i < nl; i++) jx.add(i, i);
    // with part-limb transforms, modup applies the last stages of X's inverse
    // transform and the first stages of the new limbs' forward transforms
    const int parts = ntt_parts_log(c);
    // XC and MU hold reduced fp64 patterns between these kernels (fp64
    // arithmetic, ordinary launches): no canonical form and integer
    // conversion at each hand-off
    const bool raw = raw_handoff(c);
    if (parts) run_ntt_parts(c, xc, (size_t)nl * N, count, jx, true, st, X, x_stride, false, raw);
    else run_ntt(c, xc, (size_t)nl * N, count, jx, true, st, X, x_stride);
    launch_modup(c, xc, mu, count, level, next, parts, st, raw);
    Jobs jm;
    for (int j = 0; j < nact; j++) {
        const ModUpPlan &pl = c->h_modup[(size_t)level * dnum + j];
        for (int t = 0; t < pl.ntgt; t++) jm.add(j * next + pl.tgt_e[t], pl.tgt_prime[t]);
    }
    if (parts) run_ntt_parts(c, mu, (size_t)dnum * next * N, count, jm, false, st, nullptr, 0, raw, raw);
    else run_ntt(c, mu, (size_t)dnum * next * N, count, jm, false, st);
    XC.reset();
    BufP ACC = make_buf(c, sizeof(u64) * (size_t)count * 2 * next * N);
    launch_ks_inner(c, mu, X, x_stride, key, (u64 *)ACC->p, count, level, next, nact, st, raw);
    return ACC;
}

// Relinearisation of T3 (level l > 0) followed by one modulus switch, written
// to out (level l-1): the ModDown correction and the modulus-switch correction
// are formed together in the coefficient domain and transformed once.
void relin_mod_switch(bc_ctx *c, const bc_keys *k, const CtB &t3, const CtB &out, hipStream_t st) {
    const int N = c->N, lv = t3.level, nl = lv + 1, next = nl + c->nP, count = t3.count;
    const size_t L = (size_t)nl * N;
    BufP ACC = ks_accumulate(c, k->rlk, t3.data + 2 * L, 3 * L, count, lv, st);
    u64 *acc = (u64 *)ACC->p;
    Jobs ja;  // special limbs and the top limb of both accumulators
    for (int cc = 0; cc < 2; cc++) {
        for (int t = 0; t < c->nP; t++) ja.add(cc * next + nl + t, c->nQ + t);
        ja.add(cc * next + lv, lv);
    }
    Jobs jd;  // top limb of d0 and d1 (T3 is workspace: transformed in place)
    jd.add(lv, lv);
    jd.add(nl + lv, lv);
    // with part-limb transforms the fbc kernel applies the last stages of
    // these inverse transforms and the first stages of E's forward transform
    const int parts = ntt_parts_log(c);
    // the transformed special and top limbs, d's top limbs and E pass as
    // reduced fp64 patterns (as in ks_accumulate)
    const bool raw = raw_handoff(c);
    if (parts) {
        run_ntt_parts(c, acc, (size_t)2 * next * N, count, ja, true, st, nullptr, 0, false, raw);
        run_ntt_parts(c, t3.data, 3 * L, count, jd, true, st, nullptr, 0, false, raw);
    } else {
        run_ntt(c, acc, (size_t)2 * next * N, count, ja, true, st);
        run_ntt(c, t3.data, 3 * L, count, jd, true, st);
    }
    BufP E = make_buf(c, sizeof(u64) * (size_t)count * 2 * lv * N);
    launch_relin_ms_fbc(c, acc, t3.data, 3 * L, (u64 *)E->p, count, lv, next, parts, st, raw);
    // out = (d + acc P^-1) q_l^-1 - NTT(E): fused into E's transform where the
    // schedule has such a kernel, else transform and combine separately
    NttCombine cb{};
    cb.mode = kNttRelinMs;
    cb.d = t3.data;
    cb.d_ct_stride = 3 * L;
    cb.acc = acc;
    cb.out = out.data;
    cb.level = lv;
    cb.next = next;
    const u64 ql = c->mod[lv];
    for (int i = 0; i < lv; i++) {
        const u64 q = c->mod[i];
        u64 P = 1;
        for (int t = 0; t < c->nP; t++) P = h_mulmod(P, c->mod[c->nQ + t] % q, q);
        const u64 qlinv = h_invmod(ql % q, q), pq = h_mulmod(h_invmod(P, q), qlinv, q);
        if (use_fp64(c)) {
            h_fpair(cb.w[i], qlinv, q);
            h_fpair(cb.w[i] + 2, pq, q);
        } else {
            cb.w[i][0] = qlinv;
            cb.w[i][1] = h_shoup(qlinv, q);
            cb.w[i][2] = pq;
            cb.w[i][3] = h_shoup(pq, q);
        }
    }
    LimbSet ls{};
    ls.raw_in = raw;
    ls.base = (u64 *)E->p;
    ls.poly_stride = (u64)2 * lv * N;
    ls.npoly = count;
    ls.nlimb = 2 * lv;
    for (int k = 0; k < 2 * lv; k++) {
        ls.off[k] = (int16_t)k;
        ls.prime[k] = (int16_t)(k % lv);
    }
    if (parts) {
        ntt_forward_parts_combine(c, ls, cb, st);
    } else if (!ntt_forward_combine(c, ls, cb, st)) {
        run_ntt(c, (u64 *)E->p, (size_t)2 * lv * N, count, all_limbs(2, lv), false, st);
        launch_relin_ms_combine(c, t3.data, 3 * L, acc, (u64 *)E->p, out.data, count, lv, next, st);
    }
    check_hip();
}

void key_switch(bc_ctx *c, const u64 *key, const u64 *X, size_t x_stride, int count, int level, const u64 *base0,
                const u64 *base1, size_t base_stride, u64 *out, size_t out_stride, hipStream_t st,
                bool fuse_base1 = false) {
    const int N = c->N, nl = level + 1, next = nl + c->nP;
    BufP ACC = ks_accumulate(c, key, X, x_stride, count, level, st);
    u64 *acc = (u64 *)ACC->p;
    Jobs js;
    for (int k = 0; k < 2; k++)
        for (int t = 0; t < c->nP; t++) js.add(k * next + nl + t, c->nQ + t);
    // with part-limb transforms the modulus lowering applies the last stages
    // of the special limbs' inverse transforms and the first stages of TH's
    // forward ones
    const int parts = ntt_parts_log(c);
    if (parts) run_ntt_parts(c, acc, (size_t)2 * next * N, count, js, true, st);
    else run_ntt(c, acc, (size_t)2 * next * N, count, js, true, st);
    BufP TH = make_buf(c, sizeof(u64) * (size_t)count * 2 * nl * N);
    u64 *th = (u64 *)TH->p;
    // the last step runs in TH's forward transform as it stores: TH comes out
    // of the lowering already scaled by p P^-1 and out = base + acc P^-1 -
    // NTT(TH), component 1's base the zero table when there is none.  A
    // second base is fused only for rotate-and-add: level-0 relinearisation
    // through it gave intermittent wrong results in concurrent group runs
    // (cause not found), so it keeps the separate transform and combine.
    const bool fused = !tl_rec && out_stride == (size_t)2 * nl * N && (!base1 || fuse_base1) &&
                       (parts || (c->ntt_single_pass && c->logN >= 12 && c->logN <= 15));
    launch_moddown(c, acc, th, count, level, next, parts, st, fused);
    if (fused) {
        NttCombine cb{};
        cb.mode = kNttKsCombine;
        cb.d = base0;
        cb.d_ct_stride = base_stride;
        cb.d1 = base1 ? base1 : c->zeros;
        cb.d1_ct_stride = base1 ? base_stride : 0;
        cb.d1_limb = base1 ? (u64)N : 0;
        cb.acc = acc;
        cb.out = out;
        cb.level = nl;
        cb.next = next;
        for (int i = 0; i < nl; i++) {
            const u64 q = c->mod[i];
            u64 P = 1;
            for (int t = 0; t < c->nP; t++) P = h_mulmod(P, c->mod[c->nQ + t] % q, q);
            const u64 pinv = h_invmod(P, q);
            if (use_fp64(c)) {
                h_fpair(cb.w[i], 1, q);
                h_fpair(cb.w[i] + 2, pinv, q);
            } else {
                cb.w[i][0] = 1;
                cb.w[i][1] = h_shoup(1, q);
                cb.w[i][2] = pinv;
                cb.w[i][3] = h_shoup(pinv, q);
            }
        }
        LimbSet ls{};
        ls.base = th;
        ls.poly_stride = (u64)2 * nl * N;
        ls.npoly = count;
        ls.nlimb = 2 * nl;
        for (int k = 0; k < 2 * nl; k++) {
            ls.off[k] = (int16_t)k;
            ls.prime[k] = (int16_t)(k % nl);
        }
        if (parts) ntt_forward_parts_combine(c, ls, cb, st);
        else BC_REQUIRE(ntt_forward_combine(c, ls, cb, st), BC_ERR_ARG, "key switch: no fused transform");
    } else {
        if (parts) run_ntt_parts(c, th, (size_t)2 * nl * N, count, all_limbs(2, nl), false, st);
        else run_ntt(c, th, (size_t)2 * nl * N, count, all_limbs(2, nl), false, st);
        launch_ks_combine(c, base0, base1, base_stride, acc, th, out, out_stride, count, level, next, st);
    }
    check_hip();
}

}  // namespace

// Device-to-device copy of `rows` rows of `width` words (row pitches in
// words): a recorded copy stage under the persistent executor, else a HIP copy.
static void copy_rows(const u64 *src, u64 *dst, size_t spitch, size_t dpitch, size_t width, size_t rows,
                      hipStream_t st) {
    if (tl_rec) {
        if (rows == 1) spitch = dpitch = width;
        const size_t nb = (width + kCopyBlockWords - 1) / kCopyBlockWords;
        BC_REQUIRE(nb < (1u << 30) && rows < (1u << 30), BC_ERR_ARG, "copy too large to record");
        tl_rec->add(kPkCopy, dim3((unsigned)nb, (unsigned)rows, 1), PaCopy{src, dst, spitch, dpitch, width});
        return;
    }
    if (rows == 1)
        BC_HIP(hipMemcpyAsync(dst, src, sizeof(u64) * width, hipMemcpyDeviceToDevice, st));
    else
        BC_HIP(hipMemcpy2DAsync(dst, sizeof(u64) * dpitch, src, sizeof(u64) * spitch, sizeof(u64) * width, rows,
                                hipMemcpyDeviceToDevice, st));
}

void copy_ct(const bc_ctx *c, const CtB &src, const CtB &dst, hipStream_t st) {
    BC_REQUIRE(src.count == dst.count && src.level == dst.level && src.ncomp == dst.ncomp, BC_ERR_ARG,
               "copy: shape mismatch");
    if (tl_rec) return copy_rows(src.data, dst.data, 0, 0, (size_t)src.count * src.ct_words(c->N), 1, st);
    BC_HIP(hipMemcpyAsync(dst.data, src.data, sizeof(u64) * (size_t)src.count * src.ct_words(c->N),
                          hipMemcpyDeviceToDevice, st));
}

void mod_switch(bc_ctx *c, const CtB &in, const CtB &out, hipStream_t st) {
    BC_REQUIRE(in.ncomp == 2, BC_ERR_ARG, "modulus switching takes 2-component ciphertexts");
    BC_REQUIRE(in.level >= 1, BC_ERR_LEVEL, "no prime left to drop");
    BC_REQUIRE(out.level == in.level - 1 && out.ncomp == 2 && out.count == in.count, BC_ERR_ARG,
               "modulus switch: output shape");
    const int N = c->N, lv = in.level, count = in.count;
    BufP TOP = make_buf(c, sizeof(u64) * (size_t)count * 2 * N);
    u64 *top = (u64 *)TOP->p;
    Jobs jt;  // the top limb of both components, coefficient domain, into TOP[ct][c]
    jt.add(0, lv, lv);
    jt.add(1, lv, (lv + 1) + lv);
    // with part-limb transforms the fbc kernel applies the last stages of the
    // top limbs' inverse transform and the first stages of R's forward one
    const int parts = ntt_parts_log(c);
    if (parts) run_ntt_parts(c, top, (size_t)2 * N, count, jt, true, st, in.data, in.ct_words(N));
    else run_ntt(c, top, (size_t)2 * N, count, jt, true, st, in.data, in.ct_words(N));
    BufP R = make_buf(c, sizeof(u64) * (size_t)count * 2 * lv * N);
    u64 *r = (u64 *)R->p;
    launch_ms_fbc(c, top, r, count, lv, parts, st);
    // out = (in - NTT(R)) q_l^-1: fused into R's transform where the schedule
    // has such a kernel, else transform and combine separately
    NttCombine cb{};
    cb.mode = kNttSwitch;
    cb.d = in.data;
    cb.d_ct_stride = in.ct_words(N);
    cb.out = out.data;
    cb.level = lv;
    const u64 ql = c->mod[lv];
    for (int i = 0; i < lv; i++) {
        const u64 q = c->mod[i], qlinv = h_invmod(ql % q, q);
        if (use_fp64(c)) {
            h_fpair(cb.w[i], qlinv, q);
        } else {
            cb.w[i][0] = qlinv;
            cb.w[i][1] = h_shoup(qlinv, q);
        }
    }
    LimbSet ls{};
    ls.base = r;
    ls.poly_stride = (u64)2 * lv * N;
    ls.npoly = count;
    ls.nlimb = 2 * lv;
    for (int k = 0; k < 2 * lv; k++) {
        ls.off[k] = (int16_t)k;
        ls.prime[k] = (int16_t)(k % lv);
    }
    if (parts) {
        ntt_forward_parts_combine(c, ls, cb, st);
    } else if (!ntt_forward_combine(c, ls, cb, st)) {
        run_ntt(c, r, (size_t)2 * lv * N, count, all_limbs(2, lv), false, st);
        launch_ms_combine(c, in.data, r, out.data, count, lv, st);
    }
    check_hip();
}

// Dropping k >= 2 primes: one inverse transform of every limb, the k
// single-prime switches fused per coefficient, one forward transform of the
// remaining limbs (instead of k rounds of top-limb transforms and corrections).
// Level alignment drops the top primes: every component keeps its residues
// modulo the remaining primes (one strided copy; no rescaling).  The operands
// aligned in the circuit carry noise near the modulus-switching floor, where
// a switch would not lower it.
void to_level_into(bc_ctx *c, const CtB &x, const CtB &out, hipStream_t st) {
    const int level = out.level;
    BC_REQUIRE(level >= 0 && level <= x.level, BC_ERR_LEVEL, "cannot raise a level");
    BC_REQUIRE(out.count == x.count && out.ncomp == x.ncomp, BC_ERR_ARG, "level change: output shape");
    if (x.level == level) {
        copy_ct(c, x, out, st);
        return;
    }
    const size_t limb = c->N;
    copy_rows(x.data, out.data, (x.level + 1) * limb, (level + 1) * limb, (level + 1) * limb, (size_t)x.count * x.ncomp,
              st);
}


static void check_pair(const CtB &a, const CtB &b) {
    BC_REQUIRE(b.count >= 1 && a.count % b.count == 0, BC_ERR_ARG, "second operand count must divide the first");
}

void tensor(bc_ctx *c, const CtB &a0, const CtB &b0, const CtB &out, hipStream_t st) {
    check_pair(a0, b0);
    BC_REQUIRE(a0.ncomp == 2 && b0.ncomp == 2, BC_ERR_ARG, "tensor takes 2-component ciphertexts");
    int lv = std::min(a0.level, b0.level);  // the higher operand is read at its lowest lv + 1 limbs
    BC_REQUIRE(out.ncomp == 3 && out.level == lv && out.count == a0.count, BC_ERR_ARG, "tensor: output shape");
    launch_tensor(c, a0.data, b0.data, nullptr, out.data, a0.count, b0.count, lv + 1, a0.level + 1, b0.level + 1, 0, st);
    check_hip();
}

void relin(bc_ctx *c, const bc_keys *k, const CtB &in3, const CtB &out, hipStream_t st) {
    BC_REQUIRE(in3.ncomp == 3, BC_ERR_ARG, "relinearisation takes 3-component ciphertexts");
    BC_REQUIRE(out.ncomp == 2 && out.level == in3.level && out.count == in3.count, BC_ERR_ARG,
               "relinearisation: output shape");
    const size_t L = (size_t)(in3.level + 1) * c->N;
    key_switch(c, k->rlk, in3.data + 2 * L, 3 * L, in3.count, in3.level, in3.data, in3.data + L, 3 * L, out.data,
               2 * L, st);
}

int out_level_mul(int la, int lb) {
    int lv = std::min(la, lb);
    return lv > 0 ? lv - 1 : 0;
}

// Fused-minimum HBM bytes of a batched multiplication of `count` ciphertexts
// at level lv: each operand read once, the result written once (count
// (4 (l+1) + 2 l') N 8, l' the output's limbs; an addend adds its 2 (l+1)
// limbs), and the switching key read once for the whole batch
// (2 beta_l (l+1+k) N 8).
static double mul_min_bytes(const bc_ctx *c, int count, int lv, bool addend) {
    const double nl = lv + 1, beta = lv / c->alpha + 1, nout = lv > 0 ? lv : 1;
    return 8.0 * c->N * (count * (4 * nl + 2 * nout + (addend ? 2 * nl : 0)) + 2 * beta * (nl + c->nP));
}

void mul_relin(bc_ctx *c, const bc_keys *k, const CtB &a, const CtB &b, const CtB &out, hipStream_t st) {
    check_pair(a, b);
    int lv = std::min(a.level, b.level);
    BC_REQUIRE(out.level == out_level_mul(a.level, b.level) && out.ncomp == 2 && out.count == a.count, BC_ERR_ARG,
               "multiplication: output shape");
    ProfScope ps(c, kProfMul, mul_min_bytes(c, a.count, lv, false), st);
    CtB t3 = alloc_ct(c, a.count, lv, 3);
    tensor(c, a, b, t3, st);
    if (lv == 0) {
        relin(c, k, t3, out, st);
        return;
    }
    relin_mod_switch(c, k, t3, out, st);
}

// a b + add with the addition before relinearisation and the modulus switch.
// The addend may sit above the tensor's level (it is switched down to it),
// not below.
void mul_relin_add(bc_ctx *c, const bc_keys *k, const CtB &a, const CtB &b, const CtB &add, const CtB &out,
                   hipStream_t st) {
    check_pair(a, b);
    const int lv = std::min(a.level, b.level);
    BC_REQUIRE(add.ncomp == 2 && add.count == a.count, BC_ERR_ARG, "multiply-accumulate: addend shape");
    BC_REQUIRE(add.level >= lv, BC_ERR_LEVEL, "multiply-accumulate: addend below the product's level");
    BC_REQUIRE(out.level == out_level_mul(a.level, b.level) && out.ncomp == 2 && out.count == a.count, BC_ERR_ARG,
               "multiply-accumulate: output shape");
    BC_REQUIRE(a.ncomp == 2 && b.ncomp == 2, BC_ERR_ARG, "tensor takes 2-component ciphertexts");
    ProfScope ps(c, kProfMul, mul_min_bytes(c, a.count, lv, true), st);
    // operands above lv are read at their lowest lv + 1 limbs (alignment by dropping primes)
    CtB t3 = alloc_ct(c, a.count, lv, 3);
    launch_tensor(c, a.data, b.data, add.data, t3.data, a.count, b.count, lv + 1, a.level + 1, b.level + 1,
                  add.level + 1, st);
    check_hip();
    if (lv == 0) {
        relin(c, k, t3, out, st);
        return;
    }
    relin_mod_switch(c, k, t3, out, st);
}

// Mirrors the buffers mul_relin takes: the tensor T3, then (ks_accumulate)
// the raised digits MU, the coefficient-domain copy XC and the accumulators
// ACC, then E (relinearise + switch) or, at level 0, TH (key switch).
size_t mul_relin_workspace(const bc_ctx *c, int count, int lv) {
    auto rnd = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t limb = sizeof(u64) * (size_t)c->N * count;
    const size_t nl = lv + 1, next = nl + c->nP;
    size_t t = rnd(3 * nl * limb) + rnd(c->dnum * next * limb) + rnd(nl * limb) + rnd(2 * next * limb);
    t += lv > 0 ? rnd(2 * (size_t)lv * limb) : rnd(2 * nl * limb);
    return t;
}

CtB mul(bc_ctx *c, const bc_keys *k, const CtB &a, const CtB &b, hipStream_t st) {
    CtB out = alloc_ct(c, a.count, out_level_mul(a.level, b.level), 2);
    mul_relin(c, k, a, b, out, st);
    return out;
}

u64 galois_for_step(const bc_ctx *c, int step) {
    u64 twoN = 2 * (u64)c->N;
    if (step == BC_ROW_SWAP) return twoN - 1;
    return h_powmod(5, (u64)step, twoN);
}

void rotate(bc_ctx *c, const bc_keys *k, const CtB &in, int steps, const CtB &out, hipStream_t st) {
    BC_REQUIRE(in.ncomp == 2, BC_ERR_ARG, "rotation takes 2-component ciphertexts");
    BC_REQUIRE(out.ncomp == 2 && out.level == in.level && out.count == in.count, BC_ERR_ARG, "rotation: output shape");
    int idx = -1;
    for (int i = 0; i < k->ngal; i++)
        if (k->steps[i] == steps) idx = i;
    BC_REQUIRE(idx >= 0, BC_ERR_KEY, "no rotation key for this step");
    const size_t L = (size_t)(in.level + 1) * c->N;
    CtB sig = alloc_ct(c, in.count, in.level, 2);
    launch_permute(c, in.data, sig.data, k->perm[idx], in.count, in.level + 1, 2, st);
    key_switch(c, k->gk[idx], sig.data + L, 2 * L, in.count, in.level, sig.data, nullptr, 2 * L, out.data, 2 * L, st);
}

// out = in + rotation of in: the automorphism's component 0 with in's own
// added is component 0's base of the key switch, in's component 1 that of
// component 1, so the sum costs no pass of its own (out != in)
void rotate_add(bc_ctx *c, const bc_keys *k, const CtB &in, int steps, const CtB &out, hipStream_t st) {
    BC_REQUIRE(in.ncomp == 2, BC_ERR_ARG, "rotation takes 2-component ciphertexts");
    BC_REQUIRE(out.ncomp == 2 && out.level == in.level && out.count == in.count, BC_ERR_ARG, "rotation: output shape");
    BC_REQUIRE(out.data != in.data, BC_ERR_ARG, "rotate-and-add runs out of place");
    int idx = -1;
    for (int i = 0; i < k->ngal; i++)
        if (k->steps[i] == steps) idx = i;
    BC_REQUIRE(idx >= 0, BC_ERR_KEY, "no rotation key for this step");
    const size_t L = (size_t)(in.level + 1) * c->N;
    CtB sig = alloc_ct(c, in.count, in.level, 2);
    launch_permute(c, in.data, sig.data, k->perm[idx], in.count, in.level + 1, 2, st, true);
    key_switch(c, k->gk[idx], sig.data + L, 2 * L, in.count, in.level, sig.data, in.data + L, 2 * L, out.data, 2 * L,
               st, true);
}

void add_sub(bc_ctx *c, const CtB &a0, const CtB &b0, const CtB &out, bool sub, hipStream_t st) {
    check_pair(a0, b0);
    BC_REQUIRE(a0.ncomp == b0.ncomp, BC_ERR_ARG, "component counts differ");
    int lv = std::min(a0.level, b0.level);  // the higher operand is read at its lowest lv + 1 limbs
    BC_REQUIRE(out.level == lv && out.ncomp == a0.ncomp && out.count == a0.count, BC_ERR_ARG, "add/sub: output shape");
    launch_addsub(c, a0.data, b0.data, out.data, a0.count, b0.count, lv + 1, a0.level + 1, b0.level + 1, a0.ncomp, sub,
                  st);
    check_hip();
}

CtB add(bc_ctx *c, const CtB &a, const CtB &b, hipStream_t st) {
    CtB out = alloc_ct(c, a.count, std::min(a.level, b.level), a.ncomp);
    add_sub(c, a, b, out, false, st);
    return out;
}

CtB sub(bc_ctx *c, const CtB &a, const CtB &b, hipStream_t st) {
    CtB out = alloc_ct(c, a.count, std::min(a.level, b.level), a.ncomp);
    add_sub(c, a, b, out, true, st);
    return out;
}

void mul_scalar(bc_ctx *c, const CtB &a, int64_t v, const CtB &out, hipStream_t st) {
    BC_REQUIRE(out.level == a.level && out.ncomp == a.ncomp && out.count == a.count, BC_ERR_ARG, "scalar: output shape");
    launch_mul_scalar(c, a.data, out.data, a.count, a.level + 1, a.ncomp, centred(c, v), st);
    check_hip();
}

void add_const(bc_ctx *c, const CtB &a, int64_t v, const CtB &out, hipStream_t st) {
    BC_REQUIRE(out.level == a.level && out.ncomp == a.ncomp && out.count == a.count, BC_ERR_ARG, "const: output shape");
    launch_add_const(c, a.data, out.data, a.count, a.level + 1, a.ncomp, centred(c, v), st);
    check_hip();
}

// ----------------------------------------------------------- slot encoding

namespace {

u64 least_primitive_root(u64 p) {
    std::vector<u64> fac;
    u64 n = p - 1;
    for (u64 f = 2; f * f <= n; f++)
        if (n % f == 0) {
            fac.push_back(f);
            while (n % f == 0) n /= f;
        }
    if (n > 1) fac.push_back(n);
    for (u64 g = 2; g < p; g++) {
        bool ok = true;
        for (u64 f : fac) ok = ok && h_powmod(g, (p - 1) / f, p) != 1;
        if (ok) return g;
    }
    throw Error(BC_ERR_PARAM, "no primitive root");
}

// Slot j < M/2 is the evaluation at zeta^(5^j), slot M/2 + j at zeta^(-5^j),
// zeta = g^((p-1)/2M), g the least primitive root mod p.
std::vector<u64> slot_points(const bc_ctx *c) {
    const u64 p = c->p, M = (u64)c->M, twoM = 2 * M;
    u64 zeta = h_powmod(least_primitive_root(p), (p - 1) / twoM, p);
    std::vector<u64> pts(M);
    u64 e = 1;
    for (u64 j = 0; j < M / 2; j++) {
        pts[j] = h_powmod(zeta, e, p);
        pts[M / 2 + j] = h_powmod(zeta, (twoM - e) % twoM, p);
        e = e * 5 % twoM;
    }
    return pts;
}

}  // namespace

// coefficient mu_k at x^(k N / M), mu(zeta_j) = v_j
static void encode(const bc_ctx *c, const u32 *slots, int count, u32 *m) {
    const u64 p = c->p;
    const int M = c->M, N = c->N, d = N / M;
    auto pts = slot_points(c);
    std::vector<u64> inv_pts(M);
    for (int j = 0; j < M; j++) inv_pts[j] = h_invmod(pts[j], p);
    const u64 minv = h_invmod((u64)M, p);
    std::memset(m, 0, sizeof(u32) * (size_t)count * N);
    std::vector<u64> pw(M);
    for (int ct = 0; ct < count; ct++) {
        const u32 *v = slots + (size_t)ct * M;
        for (int j = 0; j < M; j++) pw[j] = 1;
        for (int k = 0; k < M; k++) {
            u64 acc = 0;
            for (int j = 0; j < M; j++) {
                acc = (acc + (v[j] % p) * pw[j]) % p;
                pw[j] = pw[j] * inv_pts[j] % p;
            }
            m[(size_t)ct * N + (size_t)k * d] = (u32)(acc * minv % p);
        }
    }
}

void decode_slots(const bc_ctx *c, const u32 *coeffs, u32 *slots, int count) {
    const u64 p = c->p;
    const int M = c->M, N = c->N, d = N / M;
    auto pts = slot_points(c);
    for (int ct = 0; ct < count; ct++)
        for (int j = 0; j < M; j++) {
            u64 acc = 0, zk = 1;
            for (int k = 0; k < M; k++) {
                acc = (acc + (u64)coeffs[(size_t)ct * N + (size_t)k * d] * zk) % p;
                zk = zk * pts[j] % p;
            }
            slots[(size_t)ct * M + j] = (u32)acc;
        }
}

// F_{p^d} slots: slot j holds sum_k E[j][k] x^k in F_p[x]/(x^d - zeta_j), d = N/M;
// the plaintext is sum_k x^k mu_k(x^d), mu_k the slot encoding of column k
void encode_fpd(const bc_ctx *c, const u32 *elems, int count, u32 *m) {
    const u64 p = c->p;
    const int M = c->M, N = c->N, d = N / M;
    auto pts = slot_points(c);
    std::vector<u64> inv_pts(M);
    for (int j = 0; j < M; j++) inv_pts[j] = h_invmod(pts[j], p);
    const u64 minv = h_invmod((u64)M, p);
    std::memset(m, 0, sizeof(u32) * (size_t)count * N);
    std::vector<u64> col(M), pw(M);
    for (int ct = 0; ct < count; ct++)
        for (int k = 0; k < d; k++) {
            bool any = false;
            for (int j = 0; j < M; j++) {
                col[j] = elems[((size_t)ct * M + j) * d + k] % p;
                any = any || col[j];
            }
            if (!any) continue;
            for (int j = 0; j < M; j++) pw[j] = 1;
            for (int i = 0; i < M; i++) {
                u64 acc = 0;
                for (int j = 0; j < M; j++) {
                    acc = (acc + col[j] * pw[j]) % p;
                    pw[j] = pw[j] * inv_pts[j] % p;
                }
                m[(size_t)ct * N + (size_t)i * d + k] = (u32)(acc * minv % p);
            }
        }
}

// slot j's element: m mod (x^d - zeta_j), with x^(d i + k) = zeta_j^i x^k
void decode_fpd(const bc_ctx *c, const u32 *m, int count, u32 *elems) {
    const u64 p = c->p;
    const int M = c->M, N = c->N, d = N / M;
    auto pts = slot_points(c);
    std::vector<u64> acc(d);
    for (int ct = 0; ct < count; ct++)
        for (int j = 0; j < M; j++) {
            std::fill(acc.begin(), acc.end(), 0);
            u64 zi = 1;
            for (int i = 0; i < M; i++) {
                const u32 *row = m + (size_t)ct * N + (size_t)i * d;
                for (int k = 0; k < d; k++) acc[k] = (acc[k] + (row[k] % p) * zi) % p;
                zi = zi * pts[j] % p;
            }
            for (int k = 0; k < d; k++) elems[((size_t)ct * M + j) * d + k] = (u32)acc[k];
        }
}

// rotation steps r_b with 5^(r_b) = p^(2^b) mod 2N, b < log2(d): the Frobenius
// powers x -> x^(p^(2^b)) of the F_{p^d} slots (p = 1 mod 4 lies in <5>)
std::vector<int> frobenius_steps(const bc_ctx *c) {
    const u64 twoN = 2 * (u64)c->N;
    std::vector<int> log5(twoN, -1);
    u64 x = 1;
    for (int r = 0; r < c->N / 2; r++) {
        log5[x] = r;
        x = x * 5 % twoN;
    }
    std::vector<int> steps;
    for (int b = 0; (1 << b) < c->N / c->M; b++) {
        const int r = log5[h_powmod((u64)c->p % twoN, (u64)1 << b, twoN)];
        BC_REQUIRE(r >= 1, BC_ERR_PARAM, "p is not a power of 5 modulo 2N");
        steps.push_back(r);
    }
    return steps;
}

// ---------------------------------------------------------- client side

namespace {

template <class T>
BufP upload_tmp(bc_ctx *c, const T *h, size_t n, hipStream_t st) {
    BufP b = make_buf(c, sizeof(T) * n);
    BC_HIP(hipMemcpyAsync(b->p, h, sizeof(T) * n, hipMemcpyHostToDevice, st));
    return b;
}

std::vector<u32> galois_perm(const bc_ctx *c, u64 g) {
    const int N = c->N, logN = c->logN;
    const u64 twoN = 2 * (u64)N;
    std::vector<u32> perm(N);
    for (int r = 0; r < N; r++) {
        u64 e = 2 * (u64)bit_reverse(r, logN) + 1;  // position r evaluates at psi^e
        u64 eg = e * g % twoN;
        perm[r] = (u32)bit_reverse((int)((eg - 1) / 2), logN);
    }
    return perm;
}

}  // namespace

bc_keys *keygen(bc_ctx *c, const int8_t *s, const u64 *words, const int32_t *err, const int32_t *steps, int nrot) {
    BC_REQUIRE(s && words && err, BC_ERR_ARG, "keygen: null randomness");
    BC_REQUIRE(nrot >= 0 && (nrot == 0 || steps), BC_ERR_ARG, "keygen: rotation steps");
    const int N = c->N, nQ = c->nQ, nm = c->nmod, dnum = c->dnum;
    for (int r = 0; r < nrot; r++)
        BC_REQUIRE(steps[r] == BC_ROW_SWAP || (steps[r] >= 1 && steps[r] < c->N / 2), BC_ERR_ARG,
                   "rotation step out of range");
    hipStream_t st = nullptr;
    static std::atomic<uint64_t> next_uid{1};
    std::unique_ptr<bc_keys> k(new bc_keys());
    k->ctx = c;
    k->uid = next_uid.fetch_add(1);
    k->ngal = nrot;
    const size_t nwords = (size_t)nQ * N + (size_t)(1 + nrot) * dnum * nm * N;
    const size_t nerr = (size_t)N + (size_t)(1 + nrot) * dnum * N;
    BufP dw = upload_tmp(c, words, nwords, st);
    BufP de = upload_tmp(c, err, nerr, st);
    BufP ds = upload_tmp(c, s, (size_t)N, st);
    std::vector<int16_t> primes(nm);
    for (int i = 0; i < nm; i++) primes[i] = (int16_t)i;
    BufP dprimes = upload_tmp(c, primes.data(), primes.size(), st);
    const int16_t *dpr = (const int16_t *)dprimes->p;
    Jobs jall;
    for (int i = 0; i < nm; i++) jall.add(i, i);

    BC_HIP(hipMalloc(&k->s_ntt, sizeof(u64) * nm * N));
    launch_lift_small(c, nullptr, (const int8_t *)ds->p, N, nullptr, k->s_ntt, dpr, 1, nm, false, st);
    run_ntt(c, k->s_ntt, 0, 1, jall, false, st);

    BufP A = make_buf(c, sizeof(u64) * nm * N), E = make_buf(c, sizeof(u64) * nm * N);
    u64 *a = (u64 *)A->p, *e = (u64 *)E->p;
    // public key over Q
    BC_HIP(hipMalloc(&k->pk, sizeof(u64) * 2 * nQ * N));
    launch_words_mod(c, (const u64 *)dw->p, a, dpr, 1, nQ, st);
    launch_lift_small(c, (const int32_t *)de->p, nullptr, N, nullptr, e, dpr, 1, nQ, true, st);
    Jobs jq;
    for (int i = 0; i < nQ; i++) jq.add(i, i);
    run_ntt(c, a, 0, 1, jq, false, st);
    run_ntt(c, e, 0, 1, jq, false, st);
    launch_keypair(c, a, e, k->s_ntt, nullptr, nullptr, k->pk, k->pk + (size_t)nQ * N, nQ, st);

    // P mod q_i for the primes of each digit
    std::vector<u64> Pmod(nQ);
    for (int i = 0; i < nQ; i++) {
        u64 q = c->mod[i], P = 1;
        for (int t = 0; t < c->nP; t++) P = h_mulmod(P, c->mod[nQ + t] % q, q);
        Pmod[i] = P;
    }
    auto make_ksk = [&](const u64 *sprime, u64 *dst, size_t key_index) {
        for (int j = 0; j < dnum; j++) {
            const u64 *w = (const u64 *)dw->p + (size_t)nQ * N + ((key_index * dnum + j) * nm) * N;
            const int32_t *ee = (const int32_t *)de->p + N + (key_index * dnum + j) * N;
            launch_words_mod(c, w, a, dpr, 1, nm, st);
            launch_lift_small(c, ee, nullptr, N, nullptr, e, dpr, 1, nm, true, st);
            run_ntt(c, a, 0, 1, jall, false, st);
            run_ntt(c, e, 0, 1, jall, false, st);
            std::vector<u64> f(nm, 0);
            int lo = j * c->alpha, hi = std::min((j + 1) * c->alpha, nQ);
            for (int i = lo; i < hi; i++) f[i] = Pmod[i];
            u64 *k0 = dst + (size_t)j * 2 * nm * N, *k1 = k0 + (size_t)nm * N;
            launch_keypair(c, a, e, k->s_ntt, sprime, f.data(), k0, k1, nm, st);
        }
    };
    BufP S2 = make_buf(c, sizeof(u64) * nm * N);
    u64 *s2 = (u64 *)S2->p;
    launch_pmul(c, k->s_ntt, k->s_ntt, s2, nm, st);
    BC_HIP(hipMalloc(&k->rlk, sizeof(u64) * (size_t)dnum * 2 * nm * N));
    make_ksk(s2, k->rlk, 0);
    for (int r = 0; r < nrot; r++) {
        u64 g = galois_for_step(c, steps[r]);
        auto perm = galois_perm(c, g);
        u32 *dperm = nullptr;
        BC_HIP(hipMalloc(&dperm, sizeof(u32) * N));
        BC_HIP(hipMemcpy(dperm, perm.data(), sizeof(u32) * N, hipMemcpyHostToDevice));
        k->perm.push_back(dperm);
        k->steps.push_back(steps[r]);
        k->gal.push_back(g);
        launch_permute(c, k->s_ntt, s2, dperm, 1, nm, 1, st);
        u64 *gk = nullptr;
        BC_HIP(hipMalloc(&gk, sizeof(u64) * (size_t)dnum * 2 * nm * N));
        k->gk.push_back(gk);
        make_ksk(s2, gk, (size_t)(1 + r));
    }
    BC_HIP(hipStreamSynchronize(st));
    check_hip();
    return k.release();
}

// ------------------------------------------------- key export and import
// Flat little-endian format, every polynomial in the coefficient domain
// (limb-major, residues in [0, q_i)):
//   KeyBlobHeader; int32 steps[nrot]; int8 s[N] (zero-padded to a multiple
//   of 8 bytes); u64 pk[2][nQ][N]; u64 rlk[dnum][2][nQ+nP][N];
//   u64 gk[nrot][dnum][2][nQ+nP][N].
namespace {
struct KeyBlobHeader {
    char magic[4];
    uint32_t version;
    bc_params prm;
    int32_t nrot;
};
constexpr uint32_t kKeyBlobVersion = 1;

size_t key_blob_size(const bc_ctx *c, int nrot) {
    const size_t N = c->N, nm = c->nmod;
    return sizeof(KeyBlobHeader) + sizeof(int32_t) * nrot + (N + 7) / 8 * 8 +
           sizeof(u64) * (2 * c->nQ * N + (size_t)(1 + nrot) * c->dnum * 2 * nm * N);
}

// limbs [npoly][nl][N] of primes 0..nl-1 (NTT domain) -> host, coefficient domain
void download_coeff(bc_ctx *c, const u64 *dev, int npoly, int nl, int nlimb_prime_base, u64 *host, hipStream_t st) {
    const size_t words = (size_t)npoly * nl * c->N;
    BufP T = make_buf(c, sizeof(u64) * words);
    Jobs j;
    for (int i = 0; i < nl; i++) j.add(i, nlimb_prime_base + i);
    run_ntt(c, (u64 *)T->p, (size_t)nl * c->N, npoly, j, true, st, dev, (size_t)nl * c->N);
    BC_HIP(hipMemcpyAsync(host, T->p, sizeof(u64) * words, hipMemcpyDeviceToHost, st));
    BC_HIP(hipStreamSynchronize(st));
}

// host coefficient-domain limbs -> device, NTT domain (every residue checked below its prime)
void upload_ntt(bc_ctx *c, const u64 *host, int npoly, int nl, u64 *dev, hipStream_t st) {
    const size_t N = c->N;
    for (int b = 0; b < npoly; b++)
        for (int i = 0; i < nl; i++) {
            const u64 q = c->mod[i], *h = host + ((size_t)b * nl + i) * N;
            for (size_t n = 0; n < N; n++) BC_REQUIRE(h[n] < q, BC_ERR_ARG, "key import: residue out of range");
        }
    BC_HIP(hipMemcpyAsync(dev, host, sizeof(u64) * npoly * nl * N, hipMemcpyHostToDevice, st));
    Jobs j;
    for (int i = 0; i < nl; i++) j.add(i, i);
    run_ntt(c, dev, (size_t)nl * N, npoly, j, false, st);
    BC_HIP(hipStreamSynchronize(st));
}
}  // namespace

size_t keys_export(bc_ctx *c, const bc_keys *k, void *buf, size_t cap) {
    const size_t need = key_blob_size(c, k->ngal);
    if (!buf) return need;
    BC_REQUIRE(cap >= need, BC_ERR_ARG, "key export: buffer too small");
    const int N = c->N, nQ = c->nQ, nm = c->nmod, dnum = c->dnum;
    hipStream_t st = nullptr;
    char *o = (char *)buf;
    KeyBlobHeader h{};
    std::memcpy(h.magic, "BCK1", 4);
    h.version = kKeyBlobVersion;
    h.prm = c->prm;
    h.nrot = k->ngal;
    std::memcpy(o, &h, sizeof h);
    o += sizeof h;
    std::memcpy(o, k->steps.data(), sizeof(int32_t) * k->ngal);
    o += sizeof(int32_t) * k->ngal;
    // the secret's coefficients from its residues mod q_0
    std::vector<u64> s0((size_t)N);
    download_coeff(c, k->s_ntt, 1, 1, 0, s0.data(), st);
    std::memset(o, 0, (N + 7) / 8 * 8);
    const u64 q0 = c->mod[0];
    for (int n = 0; n < N; n++) o[n] = (char)(s0[n] == 0 ? 0 : s0[n] == 1 ? 1 : -1);
    (void)q0;
    o += (N + 7) / 8 * 8;
    download_coeff(c, k->pk, 2, nQ, 0, (u64 *)o, st);
    o += sizeof(u64) * 2 * nQ * N;
    auto ksk = [&](const u64 *key) {
        download_coeff(c, key, dnum * 2, nm, 0, (u64 *)o, st);
        o += sizeof(u64) * (size_t)dnum * 2 * nm * N;
    };
    ksk(k->rlk);
    for (int r = 0; r < k->ngal; r++) ksk(k->gk[r]);
    return need;
}

bc_keys *keys_import(bc_ctx *c, const void *buf, size_t size) {
    BC_REQUIRE(buf && size >= sizeof(KeyBlobHeader), BC_ERR_ARG, "key import: truncated blob");
    KeyBlobHeader h;
    std::memcpy(&h, buf, sizeof h);
    BC_REQUIRE(std::memcmp(h.magic, "BCK1", 4) == 0 && h.version == kKeyBlobVersion, BC_ERR_ARG,
               "key import: not a key blob of this version");
    BC_REQUIRE(std::memcmp(&h.prm, &c->prm, sizeof(bc_params)) == 0, BC_ERR_PARAM,
               "key import: the keys belong to another parameter set");
    BC_REQUIRE(h.nrot >= 0 && h.nrot <= 64, BC_ERR_ARG, "key import: bad rotation key count");
    BC_REQUIRE(size == key_blob_size(c, h.nrot), BC_ERR_ARG, "key import: blob size does not match its header");
    const int N = c->N, nQ = c->nQ, nm = c->nmod, dnum = c->dnum;
    hipStream_t st = nullptr;
    const char *in = (const char *)buf + sizeof h;
    std::vector<int32_t> steps(h.nrot);
    std::memcpy(steps.data(), in, sizeof(int32_t) * h.nrot);
    in += sizeof(int32_t) * h.nrot;
    for (int r = 0; r < h.nrot; r++)
        BC_REQUIRE(steps[r] == BC_ROW_SWAP || (steps[r] >= 1 && steps[r] < c->N / 2), BC_ERR_ARG,
                   "key import: rotation step out of range");
    const int8_t *sh = (const int8_t *)in;
    for (int n = 0; n < N; n++) BC_REQUIRE(sh[n] >= -1 && sh[n] <= 1, BC_ERR_ARG, "key import: secret not ternary");
    in += (N + 7) / 8 * 8;
    static std::atomic<uint64_t> next_uid{1u << 30};
    std::unique_ptr<bc_keys> k(new bc_keys());
    k->ctx = c;
    k->uid = next_uid.fetch_add(1);
    k->ngal = h.nrot;
    std::vector<int16_t> primes(nm);
    for (int i = 0; i < nm; i++) primes[i] = (int16_t)i;
    BufP dprimes = upload_tmp(c, primes.data(), primes.size(), st);
    BufP ds = upload_tmp(c, sh, (size_t)N, st);
    BC_HIP(hipMalloc(&k->s_ntt, sizeof(u64) * nm * N));
    launch_lift_small(c, nullptr, (const int8_t *)ds->p, N, nullptr, k->s_ntt, (const int16_t *)dprimes->p, 1, nm,
                      false, st);
    Jobs jall;
    for (int i = 0; i < nm; i++) jall.add(i, i);
    run_ntt(c, k->s_ntt, 0, 1, jall, false, st);
    BC_HIP(hipMalloc(&k->pk, sizeof(u64) * 2 * nQ * N));
    upload_ntt(c, (const u64 *)in, 2, nQ, k->pk, st);
    in += sizeof(u64) * 2 * nQ * N;
    const size_t kw = (size_t)dnum * 2 * nm * N;
    BC_HIP(hipMalloc(&k->rlk, sizeof(u64) * kw));
    upload_ntt(c, (const u64 *)in, dnum * 2, nm, k->rlk, st);
    in += sizeof(u64) * kw;
    for (int r = 0; r < h.nrot; r++) {
        const u64 g = galois_for_step(c, steps[r]);
        auto perm = galois_perm(c, g);
        u32 *dperm = nullptr;
        BC_HIP(hipMalloc(&dperm, sizeof(u32) * N));
        BC_HIP(hipMemcpy(dperm, perm.data(), sizeof(u32) * N, hipMemcpyHostToDevice));
        k->perm.push_back(dperm);
        k->steps.push_back(steps[r]);
        k->gal.push_back(g);
        u64 *gk = nullptr;
        BC_HIP(hipMalloc(&gk, sizeof(u64) * kw));
        k->gk.push_back(gk);
        upload_ntt(c, (const u64 *)in, dnum * 2, nm, gk, st);
        in += sizeof(u64) * kw;
    }
    BC_HIP(hipStreamSynchronize(st));
    check_hip();
    return k.release();
}

void encrypt(bc_ctx *c, const bc_keys *k, const u32 *slots, const int8_t *u, const int32_t *err, const CtB &out,
             hipStream_t st) {
    BC_REQUIRE(slots && u && err, BC_ERR_ARG, "encrypt: null input");
    std::vector<u32> m((size_t)out.count * c->N);
    encode(c, slots, out.count, m.data());
    encrypt_poly(c, k, m.data(), u, err, out, st);
}

void encrypt_poly(bc_ctx *c, const bc_keys *k, const u32 *coeffs, const int8_t *u, const int32_t *err, const CtB &out,
                  hipStream_t st) {
    BC_REQUIRE(coeffs && u && err, BC_ERR_ARG, "encrypt: null input");
    const int N = c->N, nQ = c->nQ, count = out.count;
    BC_REQUIRE(out.level == nQ - 1 && out.ncomp == 2, BC_ERR_ARG, "encrypt: output must be at the top level");
    std::vector<u32> m((size_t)count * N);
    for (size_t i = 0; i < m.size(); i++) m[i] = (u32)(coeffs[i] % (u64)c->p);
    BufP dm = upload_tmp(c, m.data(), m.size(), st);
    BufP du = upload_tmp(c, u, (size_t)count * N, st);
    BufP de = upload_tmp(c, err, (size_t)count * 2 * N, st);
    std::vector<int16_t> primes(nQ);
    for (int i = 0; i < nQ; i++) primes[i] = (int16_t)i;
    BufP dprimes = upload_tmp(c, primes.data(), primes.size(), st);
    const int16_t *dpr = (const int16_t *)dprimes->p;
    const size_t L = (size_t)nQ * N;
    BufP U = make_buf(c, sizeof(u64) * count * L), E0 = make_buf(c, sizeof(u64) * count * L),
         E1 = make_buf(c, sizeof(u64) * count * L);
    launch_lift_small(c, nullptr, (const int8_t *)du->p, N, nullptr, (u64 *)U->p, dpr, count, nQ, false, st);
    launch_lift_small(c, (const int32_t *)de->p, nullptr, 2 * N, (const u32 *)dm->p, (u64 *)E0->p, dpr, count, nQ,
                      true, st);
    launch_lift_small(c, (const int32_t *)de->p + N, nullptr, 2 * N, nullptr, (u64 *)E1->p, dpr, count, nQ, true, st);
    Jobs jq;
    for (int i = 0; i < nQ; i++) jq.add(i, i);
    run_ntt(c, (u64 *)U->p, L, count, jq, false, st);
    run_ntt(c, (u64 *)E0->p, L, count, jq, false, st);
    run_ntt(c, (u64 *)E1->p, L, count, jq, false, st);
    launch_enc_combine(c, k->pk, (u64 *)U->p, (u64 *)E0->p, (u64 *)E1->p, out.data, count, st);
    check_hip();
    // the staging buffers are released to the pool only after the stream has consumed them
    BC_HIP(hipStreamSynchronize(st));
}

void decrypt_poly(bc_ctx *c, const bc_keys *k, const CtB &in, u32 *coeffs, hipStream_t st) {
    const int N = c->N, nl = in.level + 1;
    BufP D = make_buf(c, sizeof(u64) * (size_t)in.count * nl * N);
    launch_dec_inner(c, in.data, k->s_ntt, (u64 *)D->p, in.count, nl, in.ncomp, st);
    Jobs j;
    for (int i = 0; i < nl; i++) j.add(i, i);
    run_ntt(c, (u64 *)D->p, (size_t)nl * N, in.count, j, true, st);
    BufP O = make_buf(c, sizeof(u32) * (size_t)in.count * N);
    launch_crt_decode(c, (u64 *)D->p, (u32 *)O->p, in.count, nl, st);
    check_hip();
    BC_HIP(hipMemcpyAsync(coeffs, O->p, sizeof(u32) * (size_t)in.count * N, hipMemcpyDeviceToHost, st));
    BC_HIP(hipStreamSynchronize(st));
}

void import_ct(bc_ctx *c, const u64 *host, const CtB &out, hipStream_t st) {
    BC_REQUIRE(host, BC_ERR_ARG, "import: null host buffer");
    const size_t words = (size_t)out.count * out.ct_words(c->N);
    BC_HIP(hipMemcpyAsync(out.data, host, sizeof(u64) * words, hipMemcpyHostToDevice, st));
    run_ntt(c, out.data, out.ct_words(c->N), out.count, all_limbs(out.ncomp, out.level + 1), false, st);
    check_hip();
    BC_HIP(hipStreamSynchronize(st));
}

void export_ct(bc_ctx *c, const CtB &in, u64 *host, hipStream_t st) {
    BC_REQUIRE(host, BC_ERR_ARG, "export: null host buffer");
    const size_t words = (size_t)in.count * in.ct_words(c->N);
    BufP T = make_buf(c, sizeof(u64) * words);
    run_ntt(c, (u64 *)T->p, in.ct_words(c->N), in.count, all_limbs(in.ncomp, in.level + 1), true, st, in.data,
            in.ct_words(c->N));
    check_hip();
    BC_HIP(hipMemcpyAsync(host, T->p, sizeof(u64) * words, hipMemcpyDeviceToHost, st));
    BC_HIP(hipStreamSynchronize(st));
}

}  // namespace bc
