/*
 * boostcom.h -- C ABI of the MI355X (gfx950) BGV less-than library.
 *
 * The library evaluates BoostCom's hot path -- the word-wise BGV comparison
 * (paper, Background, "Word-wise Universal FHE Scheme": integers split into
 * F_p digits, per-digit LT and EQ, lexicographic combination) -- on BGV
 * ciphertexts in RNS form (Background, "Efficient Polynomial and NTT": the
 * (L+1) x N residue matrix, NTT-based multiplication).  Ring:
 * Z_Q[x]/(x^N + 1), N a power of two, every prime q = 1 mod 2Np.  Plaintext
 * slots: M = 2^(s-1) where 2^s exactly divides p - 1 (8 for p = 17, 128 for
 * p = 257), one F_p value per slot.  Notation follows the paper's table of
 * BGV parameters (p, N, Q = q_0 ... q_L, L).
 *
 * Conventions shared by every call:
 *  - Return value: 0 on success, a negative BC_ERR_* code otherwise; no call
 *    throws.  bc_last_error() returns a message for the calling thread.  A
 *    call that fails its argument, level or noise checks launches nothing.
 *  - Ciphertext batches (bc_ctb) live in caller-owned DEVICE memory:
 *    data[count][ncomp][level+1][N] uint64 residues in [0, q_i), limb i
 *    reduced mod q_i, every limb in the NTT (evaluation) domain.  The caller
 *    sizes buffers with bc_ct_words().  Outputs must not alias inputs unless a
 *    call says otherwise; inputs are never modified.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Device work is
 *    enqueued asynchronously on it; calls returning host data synchronise it.
 *  - Host pointers are read (or written) before the call returns and stay
 *    owned by the caller.  Contexts, key sets and groups are owned by the
 *    library (created and destroyed through it).
 *  - A context is immutable after creation; calls on one context may run
 *    concurrently from several threads when they use different streams and
 *    different output buffers.  Workspace comes from a per-context pool.
 */
#ifndef BOOSTCOM_H
#define BOOSTCOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    BC_OK = 0,
    BC_ERR_ARG = -1,    /* null or malformed argument, size or shape mismatch              */
    BC_ERR_PARAM = -2,  /* impossible parameters, or objects of different parameter sets  */
    BC_ERR_LEVEL = -3,  /* no level left, or the noise estimate would exceed the budget   */
    BC_ERR_OOM = -4,    /* device or host allocation failed                                */
    BC_ERR_HIP = -5,    /* a HIP runtime call failed                                       */
    BC_ERR_KEY = -6     /* a required switching key was not generated                      */
};

/* BGV parameter set (paper, Background, "Word-wise Universal FHE Scheme":
 * the plaintext modulus p, the ring degree N and the modulus chain
 * Q = q_0 ... q_L).  Primes: the nQ largest primes below 2^bitsQ that are
 * 1 mod 2Np, in decreasing order (q_0 > ... > q_{nQ-1}); then the nP largest
 * primes below 2^bitsP with the same congruence, excluding those (special
 * primes p_0 > ... , whose product P serves key switching).  Modulus
 * switching drops the smallest remaining q.  Key switching uses dnum digits
 * of alpha = ceil(nQ/dnum) consecutive primes.  Limits: 10 <= logN <= 16,
 * p prime below 2^20, 20 <= bits <= 61, nQ + nP <= 40, 1 <= dnum <= nQ,
 * alpha <= 16, nP <= 16. */
typedef struct {
    int32_t logN;
    int32_t p;
    int32_t nQ, bitsQ;
    int32_t nP, bitsP;
    int32_t dnum;
} bc_params;

typedef struct bc_ctx bc_ctx;
typedef struct bc_keys bc_keys;

/* A batch of `count` ciphertexts at one level; see the layout above.
 * noise_bits is the library's estimate of log2 of a bound on the infinity
 * norm of [c0 + c1 s (+ c2 s^2)]_Q (paper, Background, "Word-wise Universal
 * FHE Scheme": the noise that limits the number of operations).  Every call
 * that writes a batch sets it; 0 on input means "unknown" and is taken as a
 * fresh encryption's. */
typedef struct {
    uint64_t *data;
    int32_t count;
    int32_t level;
    int32_t ncomp;
    float noise_bits;
} bc_ctb;

/* Rotation step meaning the swap of the two slot rows (x -> x^(2N-1)). */
#define BC_ROW_SWAP (-1)

/* ---------------------------------------------------------------- context */

/* Builds the prime chain, NTT twiddles and every base-conversion constant and
 * keeps them on the device (computed once; paper, The Design of BoostCom,
 * "GPU-related Optimizations": plan reuse takes data-independent work off the
 * critical path).  *out is owned by the caller until bc_ctx_destroy.
 * BC_ERR_PARAM for an impossible set (checked on the host, before any device
 * work). */
int bc_ctx_create(const bc_params *prm, bc_ctx **out);
/* Releases the caller's handle (NULL is a no-op).  The context is freed,
 * after a device wait, once its handle, every key set made from it and every
 * group that lists it are destroyed, in any order; the handle must not be
 * used after this call. */
int bc_ctx_destroy(bc_ctx *ctx);
/* moduli[nQ + nP] in the order described at bc_params (the modulus chain of
 * "Word-wise Universal FHE Scheme", then the special primes).  BC_ERR_ARG when
 * cap < nQ + nP. */
int bc_ctx_moduli(const bc_ctx *ctx, uint64_t *moduli, int32_t cap);
/* Number of plaintext slots M (the SIMD slots of "Word-wise Universal FHE
 * Scheme"), or BC_ERR_ARG for a null context. */
int bc_ctx_slots(const bc_ctx *ctx);
/* uint64 words of one ciphertext with ncomp components at `level` (the
 * (level+1) x N residue matrix of "Efficient Polynomial and NTT", per
 * component); 0 for invalid arguments. */
size_t bc_ct_words(const bc_ctx *ctx, int32_t level, int32_t ncomp);
/* Device bytes currently held by the context's workspace pool. */
size_t bc_ctx_pool_bytes(const bc_ctx *ctx);
/* Releases every cached workspace block (no call may be in flight). */
int bc_ctx_trim(bc_ctx *ctx);

/* ------------------------------------------------------------------- keys */

/* Sizes of the randomness consumed by bc_keygen for `nrot` rotation keys
 * (counts of 64-bit words and of 32-bit errors). */
int bc_keygen_rand_sizes(const bc_ctx *ctx, int32_t nrot, size_t *n_words, size_t *n_errors);

/* Key generation of BGV (paper, Background, "Word-wise Universal FHE
 * Scheme": RLWE encryption; multiplication and rotation need switching keys,
 * whose construction the paper leaves to BGV -- hybrid key switching with
 * the special primes is this library's reading) from caller-supplied
 * randomness (host arrays):
 *   s[N]        ternary secret in {-1, 0, 1};
 *   a_words     uniform 64-bit words, each reduced mod its limb's prime:
 *               public key [nQ][N], then for the relinearisation key and each
 *               rotation key (in rot_steps order) and each digit j < dnum:
 *               [nQ + nP][N];
 *   errors      small signed errors: public key [N], then per key and digit [N].
 * Produces pk = (-a s + p e, a), and switching keys
 * ksk_j = (-a_j s + p e_j + P g_j s', a_j) over Q_L * P with g_j = 1 mod the
 * primes of digit j and 0 mod all others; s' = s^2 (relinearisation) or
 * s(x^g) with g = 5^r mod 2N for each rotation step r in [1, N/2) (steps
 * from M/2 on leave the slot rows in place and act inside the F_{p^d} slots,
 * see bc_fpd_info; g = 2N - 1 for BC_ROW_SWAP; BC_ERR_ARG for other steps).  The secret stays
 * inside the key object (decryption needs it).  *out is owned by the caller
 * until bc_keys_destroy.  Synchronous. */
int bc_keygen(bc_ctx *ctx, const int8_t *s, const uint64_t *a_words, const int32_t *errors,
              const int32_t *rot_steps, int32_t nrot, bc_keys **out);
/* Waits for the device and frees the key set (NULL is a no-op); comparison
 * graphs recorded with it are dropped. */
int bc_keys_destroy(bc_keys *keys);
/* Checkpoint / resume of a key set: a flat little-endian blob (header with
 * the parameter set and the rotation steps, the ternary secret, then pk, the
 * relinearisation key and each rotation key in the COEFFICIENT domain,
 * limb-major, residues in [0, q_i)).  Export with buf == NULL stores the
 * size in *size; otherwise cap must be at least that size (BC_ERR_ARG).
 * Import checks the header (BC_ERR_PARAM for another parameter set,
 * BC_ERR_ARG for a malformed blob or out-of-range residues) and builds a key
 * set equal to the exported one.  Both synchronous. */
int bc_keys_export(bc_ctx *ctx, const bc_keys *keys, void *buf, size_t cap, size_t *size);
int bc_keys_import(bc_ctx *ctx, const void *buf, size_t size, bc_keys **out);

/* ------------------------------------------------------ client-side calls */

/* Encryption (paper, Background, "Word-wise Universal FHE Scheme": a
 * plaintext encoded into a polynomial of the slots, then encrypted).
 * Encrypts out->count slot vectors slots[count][M] (values taken mod p) at
 * the top level with public-key randomness u[count][N] (ternary) and
 * errors[count][2][N]: ct = (pk0 u + p e0 + m, pk1 u + p e1), m the slot
 * encoding (coefficient mu_k at x^(k N/M)).  out->level is set to nQ - 1,
 * out->ncomp to 2 and out->noise_bits to the fresh estimate; out->data must
 * hold bc_ct_words(nQ-1, 2) * count words. */
int bc_encrypt(bc_ctx *ctx, const bc_keys *keys, const uint32_t *slots, const int8_t *u,
               const int32_t *errors, bc_ctb *out, void *stream);

/* Decryption (same passage): [c0 + c1 s (+ c2 s^2)]_Q centred, mod p,
 * decoded to slots[count][M].  Synchronises the stream. */
int bc_decrypt(bc_ctx *ctx, const bc_keys *keys, const bc_ctb *in, uint32_t *slots, void *stream);
/* Same, returning all N plaintext coefficients in [0, p): coeffs[count][N]. */
int bc_decrypt_poly(bc_ctx *ctx, const bc_keys *keys, const bc_ctb *in, uint32_t *coeffs, void *stream);

/* Host <-> device in the COEFFICIENT domain (the inverse NTT of "Efficient
 * Polynomial and NTT" applied on export, the forward one on import):
 * host[count][ncomp][level+1][N].  Import takes out->noise_bits as given
 * (0: unknown).  Both synchronise the stream. */
int bc_export(bc_ctx *ctx, const bc_ctb *in, uint64_t *host, void *stream);
int bc_import(bc_ctx *ctx, const uint64_t *host, bc_ctb *out, void *stream);

/* ------------------------------------------------------ server-side calls */
/* Homomorphic operations of "Word-wise Universal FHE Scheme" (addition,
 * multiplication, rotation, modulus chain), each one batched launch sequence
 * over the whole residue matrix of the batch (paper, "GPU-related
 * Optimizations": element-wise work over the (L+1) x N matrix).
 * Binary calls accept b->count == a->count, or b->count dividing a->count
 * (ciphertext i of a pairs with i mod b->count of b).  An operand above the
 * lower operand's level is read at its lowest level+1 limbs: its top primes
 * are dropped without rescaling, which keeps the plaintext because every
 * q_i = 1 mod p and the noise stays below the smaller modulus.  The output
 * descriptor must have the level and component count the call produces
 * (BC_ERR_ARG otherwise); its noise_bits is set.  BC_ERR_LEVEL, before any
 * launch, when the output's noise estimate exceeds half its modulus. */

/* Tensor (a0 b0, a0 b1 + a1 b0, a1 b1): out has 3 components at min level. */
int bc_tensor(bc_ctx *ctx, const bc_ctb *a, const bc_ctb *b, bc_ctb *out, void *stream);
/* Relinearisation (key switch of c2 with the s^2 key) of a 3-component batch,
 * same level. */
int bc_relin(bc_ctx *ctx, const bc_keys *keys, const bc_ctb *in, bc_ctb *out, void *stream);
/* Modulus switch down the chain (paper: the modulus chain q_0 ... q_L):
 * drops q_level, t = [c_l p^-1]_{q_l} in (-q_l/2, q_l/2],
 * c_i' = (c_i - p t) q_l^-1.  BC_ERR_LEVEL at level 0. */
int bc_mod_switch(bc_ctx *ctx, const bc_ctb *in, bc_ctb *out, void *stream);
/* The non-scalar multiplication the comparison circuits count (paper,
 * Introduction; "Word-wise Universal FHE Scheme"): align levels, tensor,
 * relinearise, then modulus-switch one prime down unless the level is 0. */
int bc_mul_relin(bc_ctx *ctx, const bc_keys *keys, const bc_ctb *a, const bc_ctb *b, bc_ctb *out,
                 void *stream);
/* bc_mul_relin for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, same kernels, same output bytes, but no allocation of any
 * kind.  The workspace is a fixed 64 MiB device array per GPU (one copy on
 * each GPU the library runs on, held until the process ends), whose device
 * address bc_ctx_create looks up once per device.  The caller passes inputs
 * and the output as for bc_mul_relin.  Limit: (3 (l+1) + dnum (l+1+nP)
 * + (l+1) + 2 (l+1+nP) + 2 max(l,1)) N 8 count bytes, each of the five
 * buffers rounded up to 256 bytes, must fit in 64 MiB (l = the lower operand
 * level); for example one ciphertext at the top of the N = 2^15 chain
 * (14 x 50-bit + 5 x 50-bit primes, dnum 3) needs 44.25 MiB.  Larger calls
 * return BC_ERR_ARG before any launch.  Every call on one GPU uses the same
 * array and leaves its contents behind: calls on one stream are ordered, but
 * calls that overlap on one GPU (other streams, other threads, other
 * contexts) race and corrupt each other's results.  BC_ERR_HIP when the
 * array's address could not be looked up; BC_ERR_ARG when the current device
 * is not the context's. */
int bc_mul_relin_noalloc(bc_ctx *ctx, const bc_keys *keys, const bc_ctb *a, const bc_ctb *b, bc_ctb *out,
                         void *stream);
/* Rotation (paper, "Word-wise Universal FHE Scheme": rotation among the
 * homomorphic operations; the ciphertext shifting of ShiftMul/ShiftAdd) of
 * each slot row left by `steps` mod M/2 (or BC_ROW_SWAP): automorphism
 * x -> x^g, g = 5^steps mod 2N, then key switch with the matching rotation
 * key; level unchanged.  BC_ERR_KEY
 * when no rotation key was generated for `steps`. */
int bc_rotate(bc_ctx *ctx, const bc_keys *keys, const bc_ctb *in, int32_t steps, bc_ctb *out, void *stream);
/* Slot-wise addition and subtraction ("Word-wise Universal FHE Scheme";
 * the additions of the comparison circuits, Introduction). */
int bc_add(bc_ctx *ctx, const bc_ctb *a, const bc_ctb *b, bc_ctb *out, void *stream);
int bc_sub(bc_ctx *ctx, const bc_ctb *a, const bc_ctb *b, bc_ctb *out, void *stream);
/* Scalar multiplication of the circuits (paper, Introduction): multiply by c
 * in Z_p (its representative in (-p/2, p/2]). */
int bc_mul_scalar(bc_ctx *ctx, const bc_ctb *a, int32_t c, bc_ctb *out, void *stream);
/* Add the constant c in Z_p to every slot (representative in (-p/2, p/2] on
 * x^0 of c0), as the circuits' plaintext constants (EQ = 1 - Z^(p-1)). */
int bc_add_const(bc_ctx *ctx, const bc_ctb *a, int32_t c, bc_ctb *out, void *stream);

/* ---------------------------------------------------------- comparisons */
/* Word-wise comparison (paper, Background, "Word-wise Universal FHE
 * Scheme": per-digit LT and EQ over F_p, combined in lexicographic order;
 * Introduction: the univariate circuit with sqrt(p-3) + O(log p)
 * non-scalar multiplications).  Digit planes: a_digits[d] (d < ndigits <= 16,
 * most significant first) is a batch of `count` ciphertexts, all with the
 * same count, level and ncomp == 2; slot k of plane d holds digit d of
 * integer k.  The univariate circuit LT(x, y) = f(x - y), f the degree p-1
 * interpolant of [z in [(p+1)/2, p-1]], is exact for digits in
 * [0, (p-1)/2] (base (p+1)/2); it is evaluated with a Paterson-Stockmeyer
 * schedule (p - 1 a power of two: 8 multiplications for p = 17, 30 for
 * p = 257; BC_ERR_PARAM for other p).  EQ = 1 - (x - y)^(p-1).  Digits are
 * combined as LT = LT_0 + EQ_0 (LT_1 + EQ_1 (...)).
 *
 * bc_compare_levels reports the levels of the outputs for inputs at in_level
 * (max/min planes one level below LT), and BC_ERR_LEVEL when the LT circuit
 * does not fit the chain for fresh inputs (host only, no device work). */
int bc_compare_levels(const bc_ctx *ctx, int32_t in_level, int32_t ndigits, int32_t *lt_level,
                      int32_t *maxmin_level);
/* out (at the LT level): encryption of [a < b] in every slot. */
int bc_compare_lt(bc_ctx *ctx, const bc_keys *keys, int32_t ndigits, const bc_ctb *a_digits,
                  const bc_ctb *b_digits, bc_ctb *out, void *stream);
/* The comparison with max/min, the basic tasks of the paper's applications
 * (Introduction; Methodology, "Applications": min and sorting):
 * max_d = a_d + LT (b_d - a_d) and/or min_d = b_d + LT (a_d - b_d) per plane
 * (arrays of ndigits batches at the max/min level); lt_out, max_out and
 * min_out may each be NULL (at least one non-NULL).  Every step of the
 * schedule is checked against its noise budget before any launch
 * (BC_ERR_LEVEL: the circuit is deeper than the chain allows). */
int bc_compare_max_min(bc_ctx *ctx, const bc_keys *keys, int32_t ndigits, const bc_ctb *a_digits,
                       const bc_ctb *b_digits, bc_ctb *lt_out, bc_ctb *max_out, bc_ctb *min_out,
                       void *stream);

/* The bivariate circuit (paper, Introduction: the bivariate comparison
 * circuit, exact on every pair of F_p digits, about 2p multiplications;
 * Background, "Word-wise Universal FHE Scheme": the bivariate circuit
 * computes LT and EQ separately).  Digits are full-range, in [0, p-1]
 * (base p: a uint16 is two base-257 digits).  Per digit, with S = x + y and
 * Z = x - y: LT(x, y) = (p+1)/2 Z^(p-1) + sum_{k odd} Z^k g_k(S), the unique
 * interpolant of [x < y] on F_p x F_p of degree < p in S and in Z (its part
 * even in Z is (p+1)/2 Z^(p-1) because LT(x,y) + LT(y,x) = (x-y)^(p-1));
 * power ladders of S and Z (every power of S, the odd powers of Z), the g_k
 * as exact linear combinations of the S powers, one product per odd k:
 * 2p + 4 multiplications per digit for p = 257, depth log2(p-1) + 1.
 * EQ = 1 - Z^(p-1); digits are combined as for bc_compare_max_min, and so
 * are max and min.  Needs p - 1 a power of two, p < 512 and every prime
 * below 2^50 (BC_ERR_PARAM).  Arguments as for bc_compare_max_min; the
 * circuit's levels come from bc_compare_levels_circuit. */
enum { BC_CIRCUIT_UNIVARIATE = 0, BC_CIRCUIT_BIVARIATE = 1 };
int bc_compare_bivariate(bc_ctx *ctx, const bc_keys *keys, int32_t ndigits, const bc_ctb *a_digits,
                         const bc_ctb *b_digits, bc_ctb *lt_out, bc_ctb *max_out, bc_ctb *min_out, void *stream);
/* bc_compare_levels for either circuit. */
int bc_compare_levels_circuit(const bc_ctx *ctx, int32_t circuit, int32_t in_level, int32_t ndigits,
                              int32_t *lt_level, int32_t *maxmin_level);

/* Slot-packed comparison (paper, Background, "Word-wise Universal FHE
 * Scheme": the digits of one integer sit in slots of one ciphertext, and their
 * LT and EQ are combined in lexicographic order by ShiftMul -- shift the
 * ciphertext, multiply by the equality result -- and ShiftAdd -- a summation
 * done by shifting).  a, b: batches of the same count and level whose slots
 * hold base-p digits: in each slot row (M/2 slots, see bc_rotate) integer k
 * occupies slots k*l .. k*l + l - 1, most significant digit first;
 * l = digits_per_int, a power of two up to M/2 (BC_ERR_ARG).  Per-slot LT
 * and EQ by `circuit` (BC_CIRCUIT_UNIVARIATE: digits in [0, (p-1)/2];
 * BC_CIRCUIT_BIVARIATE: any digit), then log2(l) rounds with shifts
 * s = 1, 2, ..., l/2:  L <- L + E * rot(L, s),  E <- E * rot(E, s).
 * lt_out (caller-allocated, same count, level from bc_packed_levels): slot
 * k*l of every row decrypts to [a_k < b_k]; the other slots hold values of
 * no meaning.  keys must hold rotation keys for steps 1, 2, ..., l/2
 * (BC_ERR_KEY).  Depth: the digit circuit's plus log2(l) (BC_ERR_LEVEL when
 * the estimated noise would exceed a level's budget).  Runs on `stream` with
 * workspace from the context's pool; never captured into a graph. */
int bc_compare_packed(bc_ctx *ctx, const bc_keys *keys, int32_t circuit, int32_t digits_per_int, const bc_ctb *a,
                      const bc_ctb *b, bc_ctb *lt_out, void *stream);
/* Level of bc_compare_packed's output for inputs at in_level (fresh noise). */
int bc_packed_levels(const bc_ctx *ctx, int32_t circuit, int32_t in_level, int32_t digits_per_int,
                     int32_t *lt_level);

/* Tournament over small arrays of slots (same passage: comparisons between a
 * ciphertext and its own shifts).  in: a batch whose slots hold digits (one
 * digit per value, ranges as for bc_compare_packed's circuits).  For
 * window = 2^r (a power of two up to M/2, BC_ERR_ARG), r rounds with
 * s = 1, 2, ..., window/2: Y = rot(X, s), L = LT(X, Y) per slot, then
 * X <- Y + L (X - Y) (minimum) or, with want_max != 0, X <- X + L (Y - X).
 * out (same count, level from bc_tournament_levels): slot j decrypts to the
 * minimum (maximum) of slots j .. j + window - 1 of its row, cyclically; the
 * slots at multiples of `window` hold the winners of disjoint arrays of
 * `window` values.  Rotation keys for 1, 2, ..., window/2 (BC_ERR_KEY);
 * BC_ERR_LEVEL as above.  Runs on `stream`, never captured. */
int bc_tournament(bc_ctx *ctx, const bc_keys *keys, int32_t circuit, int32_t window, int32_t want_max,
                  const bc_ctb *in, bc_ctb *out, void *stream);
/* Level of bc_tournament's output for an input at in_level (fresh noise). */
int bc_tournament_levels(const bc_ctx *ctx, int32_t circuit, int32_t in_level, int32_t window, int32_t *out_level);

/* ------------------------------------------------ F_{p^d} slots */

/* Integers as elements of F_{p^d} (paper, Background, "Word-wise Universal
 * FHE Scheme": an integer is decomposed into l slots of F_{p^d}, and each
 * slot's element split into F_p digits by the mod-extract step before the
 * per-digit LT/EQ).  Over F_p, x^N + 1 is the product of the M factors
 * x^d - zeta_j (d = N/M, zeta_j the slot roots of bc_decrypt's encoding), each
 * irreducible because d is the order of p modulo 2N: slot j holds an element
 * of F_p[x]/(x^d - zeta_j), a field of p^d elements, written here in the power
 * basis 1, x, ..., x^(d-1).  The slot values of bc_encrypt are the constants.
 * The Frobenius powers x -> x^(p^(2^b)), b < log2(d), are automorphisms
 * x -> x^(5^r) with steps r in [M/2, N/2) (p = 1 mod 4 lies in <5>): their
 * rotation keys serve the extraction.
 * bc_fpd_info: *degree = d, *nsteps = log2(d), steps[0 .. log2 d) the
 * rotation steps r_b with 5^(r_b) = p^(2^b) mod 2N (cap: the array's length;
 * BC_ERR_ARG when it is too small; any pointer may be NULL).  BC_ERR_PARAM
 * when p is not a power of 5 modulo 2N. */
int bc_fpd_info(const bc_ctx *ctx, int32_t *degree, int32_t *nsteps, int32_t *steps, int32_t cap);
/* Host-side encoding: elems[count][M][d] (coordinates mod p) -> plaintext
 * coefficients coeffs[count][N] = sum_k x^k mu_k(x^d), mu_k the slot encoding
 * of coordinate k; bc_decode_fpd is its inverse (each slot's element is the
 * plaintext reduced modulo x^d - zeta_j).  Synchronous, no device work. */
int bc_encode_fpd(const bc_ctx *ctx, const uint32_t *elems, int32_t count, uint32_t *coeffs);
int bc_decode_fpd(const bc_ctx *ctx, const uint32_t *coeffs, int32_t count, uint32_t *elems);
/* Encryption of plaintext polynomials coeffs[count][N] (values taken mod p)
 * with the randomness of bc_encrypt; otherwise as bc_encrypt. */
int bc_encrypt_poly(bc_ctx *ctx, const bc_keys *keys, const uint32_t *coeffs, const int8_t *u,
                    const int32_t *errors, bc_ctb *out, void *stream);
/* The mod-extract step: for each of the ndigits coordinates k = digits[i]
 * (0 <= k < d), out holds, as ciphertexts i * in->count .. (i + 1) *
 * in->count - 1 (digit-major, at in->level, 2 components), encryptions whose
 * slot j decrypts to coordinate k of slot j's element of the input.  Computed
 * as d^-1 Tr(x^-k c): the monomial product (no noise growth), then log2(d)
 * doublings z <- z + rot(z, r_b) over the Frobenius steps (the trace over
 * the Frobenius group, which keeps the constants and removes every other
 * power of x below d), then the scalar d^-1 mod p.  out must not overlap in;
 * rotation keys for every step of bc_fpd_info (BC_ERR_KEY); BC_ERR_ARG for a
 * digit out of range or a wrong output shape; BC_ERR_LEVEL when the estimated
 * noise exceeds the input level's budget.  Runs on `stream`. */
int bc_extract_digits(bc_ctx *ctx, const bc_keys *keys, const bc_ctb *in, const int32_t *digits, int32_t ndigits,
                      bc_ctb *out, void *stream);

/* ------------------------------------------- non-power-of-two rings */

/* Transforms of the cyclotomic rings Z_q[X]/(Phi_m(X)), m odd (paper,
 * Background, "Efficient Polynomial and NTT": when the ring degree
 * n = phi(m) is not a power of two, BluesteinNTT converts polynomials between
 * coefficients and the integer DFT representation, a (L+1) x phi(m) matrix).
 * The representation of a polynomial a (degree < n) modulo prime q_i is the
 * vector of a(omega_i^k) for the k in [0, m) prime to m, ascending; omega_i is
 * the smallest x^((q_i - 1)/m), x >= 2, of order exactly m.  A plan fixes m
 * (odd, 3 <= m <= 32767 with a convolution length L -- the smallest power of
 * two >= max(2m - 1, 1024) -- of at most 2^16), `nprimes` primes (the largest
 * below 2^bits, 30 <= bits <= 61, that are 1 mod 2 L m) and everything the
 * transforms reuse: roots, the chirps TF1 = psi^(j^2) (psi = omega^((m+1)/2)),
 * the NTT of the padded chirp polynomial, the mask of the kept positions and
 * its prefix sum (the paper's branch removal: the filter is one independent
 * selective copy per position, "GPU-related Optimizations"), Phi_m and the
 * series inverse its remainder step uses.  BC_ERR_PARAM for m, nprimes or
 * bits out of range.  *out is owned by the caller until bc_bluestein_destroy. */
typedef struct bc_bluestein bc_bluestein;
int bc_bluestein_create(int32_t m, int32_t nprimes, int32_t bits, bc_bluestein **out);
/* Waits for the device and frees the plan (NULL is a no-op). */
int bc_bluestein_destroy(bc_bluestein *plan);
/* n = phi(m), the convolution length L, and the primes (nprimes words, or
 * NULL). */
int bc_bluestein_info(const bc_bluestein *plan, int32_t *n, int32_t *conv_len, uint64_t *moduli);
/* Forward (coefficients -> representation) and inverse transforms of `count`
 * polynomials: in and out are device arrays [count][nprimes][n] of canonical
 * words (residue i reduced mod prime i), distinct (BC_ERR_ARG in place).
 * Forward: the input times TF1, zero-padded to L, convolved with the chirp
 * polynomial through length-L negacyclic NTTs, folded to m words
 * (c_k = lin_k + lin_(k+m)), times TF1, filtered to the n kept positions.
 * Inverse: the values placed at their positions, the same convolution with
 * psi^-1 and m^-1, then the remainder modulo Phi_m.  Enqueued on `stream`;
 * workspace from the plan's pool.  1 <= count <= 65535. */
int bc_bluestein_forward(bc_bluestein *plan, const uint64_t *in, uint64_t *out, int32_t count, void *stream);
int bc_bluestein_inverse(bc_bluestein *plan, const uint64_t *in, uint64_t *out, int32_t count, void *stream);

/* Mixed ring sizes (paper, The Design of BoostCom, "Multi-Level
 * Heterogeneous Parallelization": independent comparisons overlapped to fill
 * the GPU; "GPU-related Optimizations": work batched onto the device at
 * once).  A group holds several contexts (e.g. N = 2^13, 2^14, 2^15), owned
 * by the caller, distinct (BC_ERR_ARG otherwise).  bc_group_compare evaluates
 * every member's comparison batch.  Per member i: keys[i], ndigits[i],
 * planes a_digits[i][0..ndigits[i]) and b_digits[i][..] as for
 * bc_compare_max_min, outputs lt_out[i] (or NULL), max_out[i] / min_out[i]
 * (arrays of ndigits[i] batches, or NULL).  Results are identical to
 * separate bc_compare_max_min calls in either mode:
 *   BC_GROUP_PERSISTENT (for members with N = 2^13, 2^14 or 2^15, every
 *   prime below 2^50 and the default transform schedule): the
 *   whole group is ONE launch of a persistent kernel that drains a device
 *   work queue.  Every kernel launch of every member's circuit becomes a
 *   stage of that queue; members are lanes (each in its own order, lanes
 *   independent, interleaved stage by stage); every transform is cut into
 *   2^13-word blocks so that one workgroup shape runs every stage of every
 *   ring size.  A stalled wait (only a library bug can cause one) ends after
 *   2 s instead of hanging, and ends every other wait of the launch; the group's next call then returns BC_ERR_HIP
 *   (for a context's own persistent comparison, BC_TUNE_PERSISTENT, so do its
 *   next persistent call and its next bc_export, bc_decrypt or bc_decrypt_poly).
 *   BC_GROUP_FORK_JOIN (the default): members run on their own streams,
 *   forked from and joined back into `stream`, each kernel its own launch.
 * In both modes the first call for a given set of buffers runs eagerly and
 * records what it launched (the persistent launch, or the whole fork/join
 * sequence) into one hipGraph; later calls replay it. */
typedef struct bc_group bc_group;
int bc_group_create(int32_t n, bc_ctx *const *ctxs, bc_group **out);
int bc_group_destroy(bc_group *g);
int bc_group_compare(bc_group *g, const bc_keys *const *keys, const int32_t *ndigits, const bc_ctb *const *a_digits,
                     const bc_ctb *const *b_digits, bc_ctb *const *lt_out, bc_ctb *const *max_out,
                     bc_ctb *const *min_out, void *stream);
enum { BC_GROUP_FORK_JOIN = 0, BC_GROUP_PERSISTENT = 1 };
/* Sets the group's mode (BC_ERR_ARG for a persistent group with a member the
 * persistent executor cannot run). */
int bc_group_set_mode(bc_group *g, int32_t mode);
/* The group's mode, and, for persistent mode, the stages, tickets and
 * resident workgroups of its last launch (any pointer may be NULL). */
int bc_group_get_mode(const bc_group *g, int32_t *mode, int32_t *stages, int32_t *tickets, int32_t *workgroups);

/* Execution mode of the comparison calls (paper, "GPU-related
 * Optimizations": whole-matrix launches instead of one per row):
 * BC_EXEC_BATCHED launches every step of the circuit once for the whole
 * batch; BC_EXEC_GRAPH additionally records the launch sequence of a (shape,
 * buffers, key set) combination into a hipGraph on its first call and
 * replays it afterwards; BC_EXEC_PER_OP runs the same kernels with one
 * ciphertext per launch (the unbatched reference path).  All modes produce
 * identical ciphertexts. */
enum { BC_EXEC_BATCHED = 0, BC_EXEC_GRAPH = 1, BC_EXEC_PER_OP = 2 };
int bc_set_exec_mode(bc_ctx *ctx, int32_t mode);

/* Tuning knobs (results never change, only speed), in the spirit of the
 * paper's plan reuse ("GPU-related Optimizations"):
 *   BC_TUNE_NTT_CHUNK_BYTES: split every batched transform into launch pairs
 *   over at most this many bytes of limbs (0 = no split), so the first pass's
 *   output is still cached when the second pass reads it.
 *   BC_TUNE_NTT_SINGLE_PASS: 1 (default) transforms a whole limb in one
 *   workgroup for N = 2^12 .. 2^15 (each word read and written once); 0 uses
 *   the two-pass column/row transform for every N.
 *   BC_TUNE_FP64: 1 (default) runs the modular arithmetic of the transforms
 *   and of the base conversions (modulus raising, the fused relinearisation
 *   and modulus switch, multi-prime switching, the polynomial's linear
 *   combinations) in exact fp64 (integers below 2^53 held in doubles) when
 *   every prime of the context is below 2^50; 0 uses 64-bit integer
 *   arithmetic.  Reading it returns 0 for a context with a prime of 2^50 or
 *   more.
 *   BC_TUNE_NTT_PARTS: nonzero (the default) lets the key-switching kernels
 *   that produce words for a forward transform apply its first one (N =
 *   2^14) or two (N = 2^15) butterfly stages themselves, so that the rest of
 *   the transform runs as independent 2^13-word parts, several per CU (only
 *   with the single-pass schedule and digits of at most 8 primes).  Results
 *   are the same bytes either way.  Reading it returns the number of folded
 *   stages in effect (0 when off or not applicable).
 *   BC_TUNE_SPLIT_STREAMS (1 .. 16, default 1): bc_compare_lt /
 *   bc_compare_max_min split the groups of a batch into this many slices,
 *   each run on a stream of the library's own (default priority) that
 *   forks from the caller's stream and joins back into it with events, so
 *   that one slice's compute-bound kernels overlap another's memory-bound
 *   ones.  Results are the same bytes; the workspace of every slice is drawn
 *   from the pool under its stream.
 *   BC_TUNE_POOL_LIMIT_BYTES: a bound on the device memory the context's
 *   workspace pool holds, blocks in use plus released blocks kept for reuse
 *   (0, the default: no bound; released blocks are then only given back by
 *   bc_ctx_trim or when an allocation fails).  When a new block would take
 *   the pool past the bound, the released blocks that were released longest
 *   ago are given back first until the new block fits under seven eighths of
 *   it (one wait for the device).  Blocks in use are never given back: a
 *   call whose own working set exceeds the bound still runs.  Set it above
 *   the working set of the batches in flight, or calls re-allocate their
 *   workspace.
 *   BC_TUNE_TEST_FAIL_ALLOC (test hook, default 0 = off): the n-th next new
 *   device allocation of the workspace pool fails, so that a caller can force
 *   BC_ERR_OOM from the host; the hook then switches itself off.
 *   BC_TUNE_PERSISTENT (default 0): 1 runs bc_compare_lt /
 *   bc_compare_max_min as ONE launch of the persistent executor (see
 *   BC_GROUP_PERSISTENT), the BC_TUNE_SPLIT_STREAMS slices of the groups as
 *   its lanes; graph mode then runs it eagerly (it is a single launch).
 *   BC_ERR_ARG where the executor cannot run the context (as for groups).
 *   BC_TUNE_MFMA (default 1): the bivariate circuit's linear combinations of
 *   the S powers (a dense 128 x 256 contraction for p = 257) run on the
 *   matrix cores as exact split-int8 products; 0 runs them in fp64 on the
 *   vector units.  Both give the same bytes.
 *   BC_TUNE_RAW_HANDOFF (default 1): with part-limb transforms and fp64
 *   arithmetic, the key-switching kernels hand their intermediate limbs to
 *   each other (raised limbs, coefficient-domain copies, the switch
 *   correction) as the bit patterns of integer-valued doubles reduced to
 *   |x| <= q/2, instead of canonical words in [0, q): one reduction instead
 *   of the canonical form and its integer conversion at every hand-off.
 *   0 keeps canonical words everywhere.  Both give the same bytes; the
 *   caller's batches always hold canonical words.
 *   BC_TUNE_MFMA_MODUP (default 0): modulus raising (the fast base
 *   conversion of each digit, with the forward transform's first stages the
 *   part-limb schedule folds into it) as an exact split-int8 contraction on
 *   the matrix cores: input residues as bytes, the constants times the fold
 *   matrix as signed base-256 digits, int32 sums recombined in fp64.  Same
 *   bytes as the fp64 kernel.  BC_ERR_ARG unless the context has fp64
 *   arithmetic, every prime above 2^33 and alpha 2^parts <= 32 (a context
 *   whose transform schedule changes afterwards runs the fp64 kernel where
 *   no table fits). */
enum {
    BC_TUNE_NTT_CHUNK_BYTES = 0,
    BC_TUNE_NTT_SINGLE_PASS = 1,
    BC_TUNE_FP64 = 2,
    BC_TUNE_POOL_LIMIT_BYTES = 3,
    BC_TUNE_NTT_PARTS = 4,
    BC_TUNE_SPLIT_STREAMS = 5,
    BC_TUNE_TEST_FAIL_ALLOC = 6,
    BC_TUNE_PERSISTENT = 7,
    BC_TUNE_MFMA = 8,
    BC_TUNE_RAW_HANDOFF = 9,
    BC_TUNE_MFMA_MODUP = 10
};
int bc_set_tuning(bc_ctx *ctx, int32_t key, int64_t value);
int bc_get_tuning(const bc_ctx *ctx, int32_t key, int64_t *value);
/* Project-written autotuner of the transform schedule (the NTT of
 * "Efficient Polynomial and NTT"): times each schedule (two-pass, two-pass in
 * cache-sized chunks, single-pass where N allows; each with fp64 and integer
 * arithmetic where the primes allow fp64) on a synthetic batch of this
 * context's shape (about 384 MB of limbs) and keeps the fastest.
 * Synchronises the stream; takes a few tens of milliseconds. */
int bc_autotune(bc_ctx *ctx, void *stream);
/* Autotuner of the whole multiplication (tensor, relinearisation and
 * modulus switch, the operation every step of the circuits repeats): times
 * bc_mul_relin at the top level on a synthetic batch of this context's shape
 * (about 512 MB of ciphertexts, at most 64) under each combination of fp64 or
 * integer arithmetic, transform schedule (single-pass, two-pass, two-pass in
 * 128 MB chunks), part-limb key-switching transforms, the reduced fp64
 * hand-off and modulus raising on the matrix cores (BC_TUNE_FP64,
 * BC_TUNE_NTT_SINGLE_PASS, BC_TUNE_NTT_CHUNK_BYTES, BC_TUNE_NTT_PARTS,
 * BC_TUNE_RAW_HANDOFF, BC_TUNE_MFMA_MODUP, where the context allows each) and
 * keeps the fastest; every combination gives the same bytes.  Needs the
 * relinearisation key of `keys`.  Synchronises the stream; takes about a
 * second at N = 2^15. */
int bc_autotune_mul(bc_ctx *ctx, const bc_keys *keys, void *stream);

/* ------------------------------------------------------------ profiling */
/* Per-kernel timing of the key-switching path (the paper measures its own
 * component breakdown, Bottleneck of uFHE Comparison).  When enabled (outside
 * graph mode), every launch of the kinds below is bracketed with HIP events
 * recorded on the stream it runs on.  bc_profile_read sums, for one kind, the
 * event-measured time (ms), the number of bracketed launches and their
 * algorithmic HBM bytes (each operand word read once, each result word
 * written once; twiddles and constants excluded):
 *   BC_PROF_NTT_FWD / _INV: whole-limb transforms, 16 N bytes per limb;
 *   BC_PROF_NTT_FWD_COMBINE: forward transforms that also apply the last
 *   step of a multiplication (relinearisation and modulus switch; 32 N bytes
 *   per limb: the limb, two operand limbs and the output) or of a modulus
 *   switch (24 N);
 *   BC_PROF_NTT_FWD_PART / _INV_PART: the part-limb transforms of key
 *   switching (BC_TUNE_NTT_PARTS; 16 N bytes per limb: the stages folded into
 *   the neighbouring kernels move no extra bytes);
 *   BC_PROF_TENSOR: the tensor (with an addend: multiply-accumulate);
 *   BC_PROF_MODUP: digit decomposition and base extension (each digit's
 *   source limbs read, its new limbs written);
 *   BC_PROF_KS_INNER: the key-switch inner product (raised limbs and the key
 *   read, two accumulators written);
 *   BC_PROF_RELIN_MS: the fused ModDown + modulus-switch correction
 *   (special and top limbs read, the correction written);
 *   BC_PROF_LINCOMB: the Paterson-Stockmeyer block combinations;
 *   BC_PROF_MUL: whole multiplications (bc_mul_relin and the circuits'
 *   multiply-accumulates, all their launches), counted at their fused
 *   minimum (4 (l+1) + 2 beta_l (l+1+k) + 2 l') 8 N bytes per ciphertext at
 *   level l (two operands read, the key read once per ciphertext, the result
 *   written; an addend adds 2 (l+1) 8 N), beta_l the active digits, k = nP,
 *   l' the result's limbs: the comparison circuit's roofline.
 * Reading synchronises on the recorded events; enabling (or disabling) clears
 * earlier records. */
enum {
    BC_PROF_NTT_FWD = 0,
    BC_PROF_NTT_INV = 1,
    BC_PROF_NTT_FWD_COMBINE = 2,
    BC_PROF_NTT_FWD_PART = 3,
    BC_PROF_NTT_INV_PART = 4,
    BC_PROF_TENSOR = 5,
    BC_PROF_MODUP = 6,
    BC_PROF_KS_INNER = 7,
    BC_PROF_RELIN_MS = 8,
    BC_PROF_LINCOMB = 9,
    BC_PROF_MUL = 10
};
int bc_profile_enable(bc_ctx *ctx, int32_t on);
int bc_profile_read(bc_ctx *ctx, int32_t kind, double *ms, int64_t *launches, double *bytes);

/* ---------------------------------------------------------- noise budget */
/* Host-only noise estimates (paper, Background, "Word-wise Universal FHE
 * Scheme": noise limits the number of operations; the modulus chain lowers
 * it), usable without a device: log2 of a bound on the infinity norm of
 * [c0 + c1 s (+ c2 s^2)]_Q after operation `op` at `level` on inputs with
 * estimates a_bits (and b_bits; 0 = a fresh encryption's):
 *   BC_NOISE_FRESH       a fresh encryption (inputs ignored);
 *   BC_NOISE_BUDGET      log2 (Q_level / 2), the most a ciphertext at
 *                        `level` may carry and still decrypt;
 *   BC_NOISE_ADD         a + b;
 *   BC_NOISE_TENSOR      the tensor of a and b;
 *   BC_NOISE_MUL         bc_mul_relin at `level` (BC_ERR_LEVEL when the
 *                        product exceeds the budget);
 *   BC_NOISE_MOD_SWITCH  dropping q_level (BC_ERR_LEVEL at level 0);
 *   BC_NOISE_ROTATE      bc_rotate at `level`.
 * The estimates assume the workloads' randomness (ternary s and u, errors of
 * deviation 3.2) and are calibrated never to fall below the exact noise of
 * the same operations.  bc_noise_compare gives the estimates of the LT and
 * (when maxmin_bits is non-NULL) max/min outputs of the comparison circuit
 * on inputs at in_level with estimate in_bits, or BC_ERR_LEVEL when a step
 * would exceed its budget.  BC_ERR_PARAM for an impossible parameter set. */
enum {
    BC_NOISE_FRESH = 0,
    BC_NOISE_BUDGET = 1,
    BC_NOISE_ADD = 2,
    BC_NOISE_TENSOR = 3,
    BC_NOISE_MUL = 4,
    BC_NOISE_MOD_SWITCH = 5,
    BC_NOISE_ROTATE = 6
};
int bc_noise_estimate(const bc_params *prm, int32_t op, int32_t level, double a_bits, double b_bits,
                      double *out_bits);
int bc_noise_compare(const bc_params *prm, int32_t in_level, double in_bits, int32_t ndigits, double *lt_bits,
                     double *maxmin_bits);
/* bc_noise_compare for either circuit (BC_CIRCUIT_UNIVARIATE or
 * BC_CIRCUIT_BIVARIATE); also reports the output levels (either pointer may
 * be NULL). */
int bc_noise_compare_circuit(const bc_params *prm, int32_t circuit, int32_t in_level, double in_bits,
                             int32_t ndigits, double *lt_bits, double *maxmin_bits, int32_t *lt_level,
                             int32_t *maxmin_level);

/* Static description of an error code, and the last error message of the
 * calling thread (valid until its next failing call). */
const char *bc_strerror(int code);
const char *bc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
