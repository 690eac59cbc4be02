/*
 * bgv_oracle.c -- plain CPU reference for the BGV less-than hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the tests, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header, table or constant
 * generator with the device library.
 *
 * What it computes (all exact integer arithmetic, every residue canonical in
 * [0, q)):
 *   - BGV over R_Q = Z_Q[x]/(x^N + 1), Q = q_0 * ... * q_L, stored in RNS form
 *     (paper, Background: "Word-wise Universal FHE Scheme" and "Efficient
 *     Polynomial and NTT": the (L+1) x phi(m) residue matrix);
 *   - every polynomial is kept in the COEFFICIENT domain; a negacyclic product
 *     is computed as twist-by-psi, textbook radix-2 cyclic NTT, pointwise
 *     product, inverse NTT, untwist (validated against the schoolbook product
 *     in the tests);
 *   - hybrid key switching: digit decomposition, fast base conversion up to
 *     Q_l * P, inner product with the switching key, and the exact division by
 *     P; modulus switching; Galois automorphisms x -> x^g.
 * The paper fixes none of the conventions (prime choice, representatives,
 * digit split); the reading used is stated at each function.
 *
 * Modular multiplication is the definition: ((unsigned __int128)a*b) % q.
 * Limb loops are spread over OpenMP threads; nothing else is tuned.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;
typedef int64_t i64;
typedef unsigned __int128 u128;

#define OR_MAXMOD 48

/* ------------------------------------------------------------------ */
/* number theory                                                       */
/* ------------------------------------------------------------------ */

u64 or_mulmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }

static u64 addmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a + b) % q); }

static u64 submod(u64 a, u64 b, u64 q) { return a >= b ? a - b : (u64)(((u128)a + q - b) % q); }

/* signed integer -> canonical residue */
static u64 smod(i64 v, u64 q) {
    if (v >= 0) return (u64)v % q;
    u64 r = (u64)(-(v + 1)) % q; /* avoids overflow at INT64_MIN */
    r = (r + 1) % q;
    return r == 0 ? 0 : q - r;
}

u64 or_powmod(u64 b, u64 e, u64 q) {
    u64 r = 1 % q;
    b %= q;
    while (e) {
        if (e & 1) r = or_mulmod(r, b, q);
        b = or_mulmod(b, b, q);
        e >>= 1;
    }
    return r;
}

/* q prime: Fermat inverse */
u64 or_invmod(u64 a, u64 q) { return or_powmod(a % q, q - 2, q); }

/* Deterministic Miller-Rabin: the first twelve primes as bases decide every
 * n < 3.18e23 (Sorenson & Webster 2015), which covers all 64-bit n. */
int or_is_prime(u64 n) {
    static const u64 bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; i++) {
        if (n == bases[i]) return 1;
        if (n % bases[i] == 0) return 0;
    }
    u64 d = n - 1;
    int r = 0;
    while ((d & 1) == 0) { d >>= 1; r++; }
    for (int i = 0; i < 12; i++) {
        u64 x = or_powmod(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int comp = 1;
        for (int k = 1; k < r; k++) {
            x = or_mulmod(x, x, n);
            if (x == n - 1) { comp = 0; break; }
        }
        if (comp) return 0;
    }
    return 1;
}

/* The `count` largest primes below 2^bits that are 1 mod `step` and not in
 * `exclude`, in decreasing order.  Returns how many were found. */
int or_gen_primes(u64 step, int bits, int count, const u64 *exclude, int nexcl, u64 *out) {
    u64 top = (bits >= 64) ? ~(u64)0 : (((u64)1 << bits) - 1);
    u64 c = ((top - 1) / step) * step + 1;
    int found = 0;
    while (found < count && c > step) {
        int skip = 0;
        for (int i = 0; i < nexcl; i++)
            if (exclude[i] == c) skip = 1;
        if (!skip && or_is_prime(c)) out[found++] = c;
        c -= step;
    }
    return found;
}

/* Smallest x >= 2 whose power x^((q-1)/2N) has order exactly 2N. */
u64 or_find_psi(u64 q, int N) {
    for (u64 x = 2; x < q; x++) {
        u64 psi = or_powmod(x, (q - 1) / (2 * (u64)N), q);
        if (or_powmod(psi, (u64)N, q) == q - 1) return psi;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* context                                                             */
/* ------------------------------------------------------------------ */

typedef struct {
    int N, logN;
    u64 p;
    int nQ, nP, dnum, alpha, nmod;
    u64 mod[OR_MAXMOD]; /* q_0 > ... > q_{nQ-1}, then special p_0 > ... > p_{nP-1} */
    u64 psi[OR_MAXMOD];
    u64 *tw[OR_MAXMOD];   /* psi^i, i < N                 */
    u64 *itw[OR_MAXMOD];  /* psi^-i, i < N                */
    u64 *om[OR_MAXMOD];   /* omega^k, omega = psi^2, k < N/2 */
    u64 *iom[OR_MAXMOD];  /* omega^-k                     */
    u64 ninv[OR_MAXMOD];  /* N^-1                         */
} or_ctx;

void or_ctx_free(or_ctx *c) {
    if (!c) return;
    for (int i = 0; i < c->nmod; i++) {
        free(c->tw[i]);
        free(c->itw[i]);
        free(c->om[i]);
        free(c->iom[i]);
    }
    free(c);
}

/* Primes: the nQ largest below 2^bitsQ, then the nP largest below 2^bitsP
 * (excluding those already taken), all congruent to 1 mod 2N*p. */
or_ctx *or_ctx_new(int logN, u64 p, int nQ, int bitsQ, int nP, int bitsP, int dnum) {
    if (logN < 1 || logN > 17 || nQ < 1 || nP < 1 || nQ + nP > OR_MAXMOD || dnum < 1 || dnum > nQ)
        return NULL;
    or_ctx *c = (or_ctx *)calloc(1, sizeof(or_ctx));
    c->logN = logN;
    c->N = 1 << logN;
    c->p = p;
    c->nQ = nQ;
    c->nP = nP;
    c->dnum = dnum;
    c->alpha = (nQ + dnum - 1) / dnum;
    c->nmod = nQ + nP;
    u64 step = 2 * (u64)c->N * p;
    if (or_gen_primes(step, bitsQ, nQ, NULL, 0, c->mod) != nQ) { free(c); return NULL; }
    if (or_gen_primes(step, bitsP, nP, c->mod, nQ, c->mod + nQ) != nP) { free(c); return NULL; }
    int N = c->N;
    for (int i = 0; i < c->nmod; i++) {
        u64 q = c->mod[i];
        u64 psi = or_find_psi(q, N);
        u64 ipsi = or_invmod(psi, q);
        u64 om = or_mulmod(psi, psi, q), iom = or_mulmod(ipsi, ipsi, q);
        c->psi[i] = psi;
        c->tw[i] = (u64 *)malloc(sizeof(u64) * N);
        c->itw[i] = (u64 *)malloc(sizeof(u64) * N);
        c->om[i] = (u64 *)malloc(sizeof(u64) * (N / 2 + 1));
        c->iom[i] = (u64 *)malloc(sizeof(u64) * (N / 2 + 1));
        u64 a = 1, b = 1;
        for (int k = 0; k < N; k++) {
            c->tw[i][k] = a;
            c->itw[i][k] = b;
            a = or_mulmod(a, psi, q);
            b = or_mulmod(b, ipsi, q);
        }
        a = 1; b = 1;
        for (int k = 0; k <= N / 2; k++) {
            c->om[i][k] = a;
            c->iom[i][k] = b;
            a = or_mulmod(a, om, q);
            b = or_mulmod(b, iom, q);
        }
        c->ninv[i] = or_invmod((u64)N, q);
    }
    return c;
}

int or_ctx_nmod(const or_ctx *c) { return c->nmod; }
void or_ctx_moduli(const or_ctx *c, u64 *out) { memcpy(out, c->mod, sizeof(u64) * c->nmod); }
u64 or_ctx_psi(const or_ctx *c, int i) { return c->psi[i]; }

/* ------------------------------------------------------------------ */
/* transforms (textbook)                                               */
/* ------------------------------------------------------------------ */

/* In-place cyclic NTT of length N with the root table w[k] = w0^k (k <= N/2):
 * bit-reversal permutation followed by log2 N radix-2 Cooley-Tukey passes.
 * Output position k holds sum_i a_i w0^(i k). */
static void cyclic_ntt(u64 *a, int N, const u64 *w, u64 q) {
    for (int i = 1, j = 0; i < N; i++) {
        int bit = N >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { u64 t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    for (int len = 2; len <= N; len <<= 1) {
        int half = len >> 1, stride = N / len;
        for (int i = 0; i < N; i += len)
            for (int j = 0; j < half; j++) {
                u64 u = a[i + j];
                u64 v = or_mulmod(a[i + j + half], w[j * stride], q);
                a[i + j] = addmod(u, v, q);
                a[i + j + half] = submod(u, v, q);
            }
    }
}

/* Negacyclic evaluation: position k holds a(psi^(2k+1)). */
void or_ntt_forward(const or_ctx *c, int m, u64 *a) {
    u64 q = c->mod[m];
    for (int i = 0; i < c->N; i++) a[i] = or_mulmod(a[i], c->tw[m][i], q);
    cyclic_ntt(a, c->N, c->om[m], q);
}

void or_ntt_inverse(const or_ctx *c, int m, u64 *a) {
    u64 q = c->mod[m];
    cyclic_ntt(a, c->N, c->iom[m], q);
    for (int i = 0; i < c->N; i++) a[i] = or_mulmod(or_mulmod(a[i], c->ninv[m], q), c->itw[m][i], q);
}

/* out = a * b mod (x^N + 1, q_m), via the transforms above. */
void or_negacyclic_mul(const or_ctx *c, int m, const u64 *a, const u64 *b, u64 *out) {
    int N = c->N;
    u64 q = c->mod[m];
    u64 *fa = (u64 *)malloc(sizeof(u64) * N), *fb = (u64 *)malloc(sizeof(u64) * N);
    memcpy(fa, a, sizeof(u64) * N);
    memcpy(fb, b, sizeof(u64) * N);
    or_ntt_forward(c, m, fa);
    or_ntt_forward(c, m, fb);
    for (int i = 0; i < N; i++) fa[i] = or_mulmod(fa[i], fb[i], q);
    or_ntt_inverse(c, m, fa);
    memcpy(out, fa, sizeof(u64) * N);
    free(fa);
    free(fb);
}

/* Schoolbook negacyclic product: x^i * x^j = x^(i+j) if i+j < N, else -x^(i+j-N). */
void or_schoolbook_negacyclic(const u64 *a, const u64 *b, u64 *out, int N, u64 q) {
    for (int k = 0; k < N; k++) out[k] = 0;
    for (int i = 0; i < N; i++)
        for (int j = 0; j < N; j++) {
            u64 t = or_mulmod(a[i], b[j], q);
            int k = i + j;
            if (k < N) out[k] = addmod(out[k], t, q);
            else out[k - N] = submod(out[k - N], t, q);
        }
}

/* ------------------------------------------------------------------ */
/* helpers on residue polynomials                                      */
/* ------------------------------------------------------------------ */

/* Prime index of limb e of a polynomial at level l, in the basis
 * q_0..q_l (extended: followed by the nP special primes). */
static int ext_prime(const or_ctx *c, int level, int e) { return e <= level ? e : c->nQ + (e - level - 1); }

static void lift_small(const or_ctx *c, int m, const int32_t *v, u64 *out) {
    for (int i = 0; i < c->N; i++) out[i] = smod((i64)v[i], c->mod[m]);
}

/* Digit j at level l: primes [j*alpha, min((j+1)*alpha, l+1)); returns 0 if empty. */
static int digit_range(const or_ctx *c, int level, int j, int *lo, int *hi) {
    *lo = j * c->alpha;
    *hi = (j + 1) * c->alpha;
    if (*hi > c->nQ) *hi = c->nQ;
    if (*hi > level + 1) *hi = level + 1;
    return *lo < *hi;
}

/* ------------------------------------------------------------------ */
/* key generation                                                      */
/* ------------------------------------------------------------------ */

/* Switching key for s' (coefficient residues over all nmod primes):
 * ksk_j = (-a_j s + p e_j + P g_j s', a_j), g_j = 1 mod the primes of digit j
 * and 0 mod every other prime (the special primes included). */
static void make_ksk(const or_ctx *c, const u64 *sres, const u64 *sp, const u64 *a_words, const int32_t *e,
                     u64 *ksk) {
    int N = c->N, nm = c->nmod;
    for (int j = 0; j < c->dnum; j++) {
        int lo, hi;
        digit_range(c, c->nQ - 1, j, &lo, &hi);
        const u64 *aw = a_words + (size_t)j * nm * N;
        const int32_t *ej = e + (size_t)j * N;
        u64 *k0 = ksk + ((size_t)j * 2 + 0) * nm * N;
        u64 *k1 = ksk + ((size_t)j * 2 + 1) * nm * N;
#pragma omp parallel for schedule(dynamic)
        for (int m = 0; m < nm; m++) {
            u64 q = c->mod[m];
            u64 *a = k1 + (size_t)m * N;
            u64 *as = (u64 *)malloc(sizeof(u64) * N);
            for (int i = 0; i < N; i++) a[i] = aw[(size_t)m * N + i] % q;
            or_negacyclic_mul(c, m, a, sres + (size_t)m * N, as);
            u64 Pm = 1; /* P mod q_m */
            for (int t = 0; t < c->nP; t++) Pm = or_mulmod(Pm, c->mod[c->nQ + t] % q, q);
            int in_digit = (m >= lo && m < hi);
            for (int i = 0; i < N; i++) {
                u64 v = submod(0, as[i], q);
                v = addmod(v, or_mulmod(c->p % q, smod(ej[i], q), q), q);
                if (in_digit) v = addmod(v, or_mulmod(Pm, sp[(size_t)m * N + i], q), q);
                k0[(size_t)m * N + i] = v;
            }
            free(as);
        }
    }
}

/* x -> x^g on a coefficient vector mod q. */
static void automorph_limb(const u64 *a, u64 *out, int N, i64 g, u64 q) {
    i64 twoN = 2 * (i64)N;
    for (int i = 0; i < N; i++) {
        i64 j = ((i64)i * g) % twoN;
        if (j < N) out[j] = a[i];
        else out[j - N] = submod(0, a[i], q);
    }
}

/*
 * Randomness layout (shared with the device library's key generator):
 *   a_words: pk [nQ][N], then for key k (relin, gal_0, gal_1, ...) and digit j:
 *            [nQ+nP][N];
 *   e:       pk [N], then per key k and digit j: [N].
 * Outputs (coefficient domain):
 *   sk [nmod][N]; pk [2][nQ][N]; rlk [dnum][2][nmod][N];
 *   gk [ngal][dnum][2][nmod][N]  (for s' = s(x^g)).
 */
void or_keygen(const or_ctx *c, const int8_t *s, const u64 *a_words, const int32_t *e, const i64 *gal, int ngal,
               u64 *sk, u64 *pk, u64 *rlk, u64 *gk) {
    int N = c->N, nm = c->nmod, nQ = c->nQ;
    for (int m = 0; m < nm; m++)
        for (int i = 0; i < N; i++) sk[(size_t)m * N + i] = smod((i64)s[i], c->mod[m]);
    /* public key */
#pragma omp parallel for
    for (int m = 0; m < nQ; m++) {
        u64 q = c->mod[m];
        u64 *a = pk + ((size_t)nQ + m) * N;
        u64 *as = (u64 *)malloc(sizeof(u64) * N);
        for (int i = 0; i < N; i++) a[i] = a_words[(size_t)m * N + i] % q;
        or_negacyclic_mul(c, m, a, sk + (size_t)m * N, as);
        for (int i = 0; i < N; i++)
            pk[(size_t)m * N + i] = addmod(submod(0, as[i], q), or_mulmod(c->p % q, smod(e[i], q), q), q);
        free(as);
    }
    const u64 *aw = a_words + (size_t)nQ * N;
    const int32_t *ew = e + N;
    size_t kwords = (size_t)c->dnum * nm * N, kerr = (size_t)c->dnum * N;
    /* relinearisation key: s' = s^2 */
    u64 *s2 = (u64 *)malloc(sizeof(u64) * nm * N);
#pragma omp parallel for
    for (int m = 0; m < nm; m++) or_negacyclic_mul(c, m, sk + (size_t)m * N, sk + (size_t)m * N, s2 + (size_t)m * N);
    make_ksk(c, sk, s2, aw, ew, rlk);
    /* Galois keys: s' = s(x^g) */
    for (int k = 0; k < ngal; k++) {
        for (int m = 0; m < nm; m++) automorph_limb(sk + (size_t)m * N, s2 + (size_t)m * N, N, gal[k], c->mod[m]);
        make_ksk(c, sk, s2, aw + (size_t)(k + 1) * kwords, ew + (size_t)(k + 1) * kerr,
                 gk + (size_t)k * 2 * kwords);
    }
    free(s2);
}

/* ------------------------------------------------------------------ */
/* encryption / decryption                                             */
/* ------------------------------------------------------------------ */

/* ct = (pk0 u + p e0 + m, pk1 u + p e1) mod Q_L; m coefficients in [0, p). */
void or_encrypt(const or_ctx *c, const u64 *pk, const uint32_t *msg, const int8_t *u, const int32_t *e0,
                const int32_t *e1, u64 *out) {
    int N = c->N, nQ = c->nQ;
#pragma omp parallel for
    for (int m = 0; m < nQ; m++) {
        u64 q = c->mod[m];
        u64 *ur = (u64 *)malloc(sizeof(u64) * N), *t = (u64 *)malloc(sizeof(u64) * N);
        for (int i = 0; i < N; i++) ur[i] = smod((i64)u[i], q);
        u64 pq = c->p % q;
        or_negacyclic_mul(c, m, pk + (size_t)m * N, ur, t);
        for (int i = 0; i < N; i++)
            out[(size_t)m * N + i] = addmod(addmod(t[i], or_mulmod(pq, smod(e0[i], q), q), q), (u64)msg[i] % q, q);
        or_negacyclic_mul(c, m, pk + ((size_t)nQ + m) * N, ur, t);
        for (int i = 0; i < N; i++)
            out[((size_t)nQ + m) * N + i] = addmod(t[i], or_mulmod(pq, smod(e1[i], q), q), q);
        free(ur);
        free(t);
    }
}

/* out[i] = c0 + c1 s (+ c2 s^2) mod q_i, i <= level (coefficient domain). */
void or_decrypt_residues(const or_ctx *c, const u64 *sk, const u64 *ct, int level, int ncomp, u64 *out) {
    int N = c->N, nl = level + 1;
#pragma omp parallel for
    for (int m = 0; m < nl; m++) {
        u64 q = c->mod[m];
        const u64 *s = sk + (size_t)m * N;
        u64 *t = (u64 *)malloc(sizeof(u64) * N), *sp = (u64 *)malloc(sizeof(u64) * N);
        for (int i = 0; i < N; i++) out[(size_t)m * N + i] = ct[(size_t)m * N + i];
        memcpy(sp, s, sizeof(u64) * N);
        for (int k = 1; k < ncomp; k++) {
            or_negacyclic_mul(c, m, ct + ((size_t)k * nl + m) * N, sp, t);
            for (int i = 0; i < N; i++) out[(size_t)m * N + i] = addmod(out[(size_t)m * N + i], t[i], q);
            if (k + 1 < ncomp) or_negacyclic_mul(c, m, sp, s, sp);
        }
        free(t);
        free(sp);
    }
}

/* ------------------------------------------------------------------ */
/* ring operations on ciphertexts ([ncomp][level+1][N])               */
/* ------------------------------------------------------------------ */

void or_add(const or_ctx *c, const u64 *a, const u64 *b, int level, int ncomp, u64 *out) {
    int N = c->N, nl = level + 1;
    for (int k = 0; k < ncomp; k++)
        for (int m = 0; m < nl; m++)
            for (int i = 0; i < N; i++) {
                size_t x = ((size_t)k * nl + m) * N + i;
                out[x] = addmod(a[x], b[x], c->mod[m]);
            }
}

void or_sub(const or_ctx *c, const u64 *a, const u64 *b, int level, int ncomp, u64 *out) {
    int N = c->N, nl = level + 1;
    for (int k = 0; k < ncomp; k++)
        for (int m = 0; m < nl; m++)
            for (int i = 0; i < N; i++) {
                size_t x = ((size_t)k * nl + m) * N + i;
                out[x] = submod(a[x], b[x], c->mod[m]);
            }
}

/* multiply every residue by the signed integer s */
void or_mul_scalar(const or_ctx *c, const u64 *a, int level, int ncomp, i64 s, u64 *out) {
    int N = c->N, nl = level + 1;
    for (int k = 0; k < ncomp; k++)
        for (int m = 0; m < nl; m++) {
            u64 sv = smod(s, c->mod[m]);
            for (int i = 0; i < N; i++) {
                size_t x = ((size_t)k * nl + m) * N + i;
                out[x] = or_mulmod(a[x], sv, c->mod[m]);
            }
        }
}

/* add the signed integer s to the constant coefficient of component 0 */
void or_add_const(const or_ctx *c, const u64 *a, int level, int ncomp, i64 s, u64 *out) {
    int N = c->N, nl = level + 1;
    memcpy(out, a, sizeof(u64) * (size_t)ncomp * nl * N);
    for (int m = 0; m < nl; m++) out[(size_t)m * N] = addmod(out[(size_t)m * N], smod(s, c->mod[m]), c->mod[m]);
}

/* (a0 b0, a0 b1 + a1 b0, a1 b1) */
void or_tensor(const or_ctx *c, const u64 *a, const u64 *b, int level, u64 *out) {
    int N = c->N, nl = level + 1;
#pragma omp parallel for
    for (int m = 0; m < nl; m++) {
        u64 q = c->mod[m];
        const u64 *a0 = a + (size_t)m * N, *a1 = a + ((size_t)nl + m) * N;
        const u64 *b0 = b + (size_t)m * N, *b1 = b + ((size_t)nl + m) * N;
        u64 *d0 = out + (size_t)m * N, *d1 = out + ((size_t)nl + m) * N, *d2 = out + ((size_t)2 * nl + m) * N;
        u64 *t = (u64 *)malloc(sizeof(u64) * N);
        or_negacyclic_mul(c, m, a0, b0, d0);
        or_negacyclic_mul(c, m, a0, b1, d1);
        or_negacyclic_mul(c, m, a1, b0, t);
        for (int i = 0; i < N; i++) d1[i] = addmod(d1[i], t[i], q);
        or_negacyclic_mul(c, m, a1, b1, d2);
        free(t);
    }
}

/* Drop q_level: t = [c_level * p^-1]_{q_level} lifted to (-q_level/2, q_level/2],
 * c'_i = (c_i - p t) * q_level^-1 mod q_i.  Output at level-1. */
void or_mod_switch(const or_ctx *c, const u64 *a, int level, int ncomp, u64 *out) {
    int N = c->N, nl = level + 1, nlo = level;
    u64 ql = c->mod[level];
    u64 pinv = or_invmod(c->p % ql, ql);
    for (int k = 0; k < ncomp; k++) {
        const u64 *top = a + ((size_t)k * nl + level) * N;
        for (int m = 0; m < nlo; m++) {
            u64 q = c->mod[m];
            u64 qlinv = or_invmod(ql % q, q);
            for (int i = 0; i < N; i++) {
                u64 t = or_mulmod(top[i], pinv, ql);
                i64 tc = (t > (ql - 1) / 2) ? (i64)t - (i64)ql : (i64)t;
                u64 pt = or_mulmod(c->p % q, smod(tc, q), q);
                u64 v = submod(a[((size_t)k * nl + m) * N + i], pt, q);
                out[((size_t)k * nlo + m) * N + i] = or_mulmod(v, qlinv, q);
            }
        }
    }
}

/* Fast base conversion of digit j of x (level l, limbs 0..l) to the extended
 * basis q_0..q_l, p_0..p_{nP-1}.  With D the digit's primes and
 * Qhat_i = prod_{i' in D, i' != i} q_i':
 *   y_i = [x_i * Qhat_i^-1]_{q_i} in [0, q_i),   u_m = sum_i y_i * Qhat_i mod q_m,
 * and the digit's own limbs are copied exactly. */
void or_modup(const or_ctx *c, const u64 *x, int level, int j, u64 *out) {
    int N = c->N, lo, hi, next = level + 1 + c->nP;
    if (!digit_range(c, level, j, &lo, &hi)) return;
    int a = hi - lo;
    u64 qhinv[OR_MAXMOD];
    for (int i = lo; i < hi; i++) {
        u64 q = c->mod[i], prod = 1;
        for (int t = lo; t < hi; t++)
            if (t != i) prod = or_mulmod(prod, c->mod[t] % q, q);
        qhinv[i - lo] = or_invmod(prod, q);
    }
#pragma omp parallel for
    for (int e = 0; e < next; e++) {
        int m = ext_prime(c, level, e);
        u64 q = c->mod[m];
        if (e >= lo && e < hi) {
            memcpy(out + (size_t)e * N, x + (size_t)e * N, sizeof(u64) * N);
            continue;
        }
        u64 qhat[OR_MAXMOD];
        for (int i = lo; i < hi; i++) {
            u64 prod = 1;
            for (int t = lo; t < hi; t++)
                if (t != i) prod = or_mulmod(prod, c->mod[t] % q, q);
            qhat[i - lo] = prod;
        }
        for (int n = 0; n < N; n++) {
            u64 acc = 0;
            for (int i = 0; i < a; i++) {
                u64 y = or_mulmod(x[(size_t)(lo + i) * N + n], qhinv[i], c->mod[lo + i]);
                acc = addmod(acc, or_mulmod(y, qhat[i], q), q);
            }
            out[(size_t)e * N + n] = acc;
        }
    }
}

/* Exact division by P of the extended polynomial acc (limbs q_0..q_l then
 * the special primes), keeping the plaintext:
 *   v_j = [acc_{p_j} * p^-1 * Phat_j^-1]_{p_j},  t_i = sum_j v_j * Phat_j mod q_i,
 *   out_i = (acc_i - p t_i) * P^-1 mod q_i. */
void or_moddown(const or_ctx *c, const u64 *acc, int level, u64 *out) {
    int N = c->N, nP = c->nP, nQ = c->nQ;
    u64 vfac[OR_MAXMOD];
    for (int j = 0; j < nP; j++) {
        u64 pj = c->mod[nQ + j], prod = 1;
        for (int t = 0; t < nP; t++)
            if (t != j) prod = or_mulmod(prod, c->mod[nQ + t] % pj, pj);
        vfac[j] = or_mulmod(or_invmod(c->p % pj, pj), or_invmod(prod, pj), pj);
    }
#pragma omp parallel for
    for (int i = 0; i <= level; i++) {
        u64 q = c->mod[i];
        u64 phat[OR_MAXMOD], P = 1;
        for (int j = 0; j < nP; j++) {
            u64 prod = 1;
            for (int t = 0; t < nP; t++)
                if (t != j) prod = or_mulmod(prod, c->mod[nQ + t] % q, q);
            phat[j] = prod;
            P = or_mulmod(P, c->mod[nQ + j] % q, q);
        }
        u64 Pinv = or_invmod(P, q);
        for (int n = 0; n < N; n++) {
            u64 t = 0;
            for (int j = 0; j < nP; j++) {
                u64 pj = c->mod[nQ + j];
                u64 v = or_mulmod(acc[(size_t)(level + 1 + j) * N + n], vfac[j], pj);
                t = addmod(t, or_mulmod(v % q, phat[j], q), q);
            }
            u64 d = submod(acc[(size_t)i * N + n], or_mulmod(c->p % q, t, q), q);
            out[(size_t)i * N + n] = or_mulmod(d, Pinv, q);
        }
    }
}

/* Hybrid key switch of d (level l, coefficient domain) with ksk
 * [dnum][2][nmod][N]: returns (ks0, ks1) at level l with
 * ks0 + ks1 s = d s' + small noise (mod Q_l). */
void or_key_switch(const or_ctx *c, const u64 *ksk, const u64 *d, int level, u64 *out) {
    int N = c->N, nm = c->nmod, next = level + 1 + c->nP;
    u64 *acc = (u64 *)calloc((size_t)2 * next * N, sizeof(u64));
    u64 *u = (u64 *)malloc(sizeof(u64) * next * N);
    for (int j = 0; j < c->dnum; j++) {
        int lo, hi;
        if (!digit_range(c, level, j, &lo, &hi)) continue;
        or_modup(c, d, level, j, u);
        for (int k = 0; k < 2; k++) {
            const u64 *key = ksk + ((size_t)j * 2 + k) * nm * N;
#pragma omp parallel for
            for (int e = 0; e < next; e++) {
                int m = ext_prime(c, level, e);
                u64 *t = (u64 *)malloc(sizeof(u64) * N);
                or_negacyclic_mul(c, m, u + (size_t)e * N, key + (size_t)m * N, t);
                u64 *dst = acc + ((size_t)k * next + e) * N;
                for (int i = 0; i < N; i++) dst[i] = addmod(dst[i], t[i], c->mod[m]);
                free(t);
            }
        }
    }
    for (int k = 0; k < 2; k++) or_moddown(c, acc + (size_t)k * next * N, level, out + (size_t)k * (level + 1) * N);
    free(u);
    free(acc);
}

/* (d0, d1, d2) -> (d0 + ks0, d1 + ks1) with the relinearisation key. */
void or_relin(const or_ctx *c, const u64 *rlk, const u64 *ct3, int level, u64 *out) {
    int N = c->N, nl = level + 1;
    u64 *ks = (u64 *)malloc(sizeof(u64) * 2 * nl * N);
    or_key_switch(c, rlk, ct3 + (size_t)2 * nl * N, level, ks);
    or_add(c, ct3, ks, level, 2, out);
    free(ks);
}

/* x -> x^g on every component and limb */
void or_automorphism(const or_ctx *c, const u64 *a, int level, int ncomp, i64 g, u64 *out) {
    int N = c->N, nl = level + 1;
    for (int k = 0; k < ncomp; k++)
        for (int m = 0; m < nl; m++)
            automorph_limb(a + ((size_t)k * nl + m) * N, out + ((size_t)k * nl + m) * N, N, g, c->mod[m]);
}

/* (sigma(c0), sigma(c1)) key-switched from s(x^g) back to s. */
void or_rotate(const or_ctx *c, const u64 *gk, const u64 *ct, int level, i64 g, u64 *out) {
    int N = c->N, nl = level + 1;
    u64 *sg = (u64 *)malloc(sizeof(u64) * 2 * nl * N);
    u64 *ks = (u64 *)malloc(sizeof(u64) * 2 * nl * N);
    or_automorphism(c, ct, level, 2, g, sg);
    or_key_switch(c, gk, sg + (size_t)nl * N, level, ks);
    for (int m = 0; m < nl; m++)
        for (int i = 0; i < N; i++) {
            size_t x0 = (size_t)m * N + i, x1 = ((size_t)nl + m) * N + i;
            out[x0] = addmod(sg[x0], ks[x0], c->mod[m]);
            out[x1] = ks[x1];
        }
    free(sg);
    free(ks);
}

/* ------------------------------------------------------------------ */
/* cyclotomic rings of odd order m (the non-power-of-two rings)        */
/* ------------------------------------------------------------------ */

/* Smallest x >= 2 whose power x^((q-1)/m) has order exactly m (m | q - 1):
 * w^(m/r) != 1 for every prime r dividing m. */
u64 or_find_root_m(u64 q, u64 m) {
    u64 fac[32];
    int nf = 0;
    u64 t = m;
    for (u64 r = 2; r * r <= t; r++)
        if (t % r == 0) {
            fac[nf++] = r;
            while (t % r == 0) t /= r;
        }
    if (t > 1) fac[nf++] = t;
    for (u64 x = 2; x < q; x++) {
        u64 w = or_powmod(x, (q - 1) / m, q);
        int ok = w != 1 || m == 1;
        for (int i = 0; i < nf && ok; i++)
            if (or_powmod(w, m / fac[i], q) == 1) ok = 0;
        if (ok) return w;
    }
    return 0;
}

/* Horner evaluation: out[k] = sum_{i<n} a[i] x[k]^i mod q. */
void or_poly_eval(const u64 *a, int n, const u64 *x, int npts, u64 q, u64 *out) {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < npts; k++) {
        u64 acc = 0;
        for (int i = n - 1; i >= 0; i--) acc = addmod(or_mulmod(acc, x[k], q), a[i], q);
        out[k] = acc;
    }
}

/* Remainder of b (length nb) modulo the monic phi of degree n (phi[0..n],
 * signed coefficients) over Z_q, by long division; out has n words. */
void or_poly_mod_monic(const u64 *b, int nb, const i64 *phi, int n, u64 q, u64 *out) {
    u64 *r = (u64 *)malloc(sizeof(u64) * (size_t)(nb > n ? nb : n));
    for (int i = 0; i < nb; i++) r[i] = b[i] % q;
    for (int i = nb; i < n; i++) r[i] = 0;
    for (int top = nb - 1; top >= n; top--) {
        const u64 c = r[top];
        if (!c) continue;
        /* r -= c X^(top-n) phi */
        for (int j = 0; j <= n; j++) {
            if (!phi[j]) continue;
            const u64 t = or_mulmod(c, smod(phi[j], q), q);
            r[top - n + j] = submod(r[top - n + j], t, q);
        }
    }
    memcpy(out, r, sizeof(u64) * n);
    free(r);
}

/* Schoolbook product of a and b (n coefficients each) modulo phi (monic,
 * degree n) over Z_q. */
void or_cyclo_mul(const u64 *a, const u64 *b, int n, const i64 *phi, u64 q, u64 *out) {
    const int np = 2 * n - 1;
    u64 *p = (u64 *)malloc(sizeof(u64) * (size_t)np);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < np; k++) {
        u64 acc = 0;
        const int lo = k - (n - 1) > 0 ? k - (n - 1) : 0, hi = k < n - 1 ? k : n - 1;
        for (int i = lo; i <= hi; i++) acc = addmod(acc, or_mulmod(a[i], b[k - i], q), q);
        p[k] = acc;
    }
    or_poly_mod_monic(p, np, phi, n, q, out);
    free(p);
}
