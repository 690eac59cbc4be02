// ops.h -- BGV operations on device batches (host orchestration).
#pragma once

#include "kernels.h"

namespace bc {

// Caller-provided workspace carved front to back (allocation-free calls):
// while a thread has one installed, every workspace buffer of its operations
// comes from it instead of the pool, and nothing is returned until the call
// ends.
struct Arena {
    char *base;
    size_t cap, used = 0;
    void *take(size_t bytes) {
        bytes = (bytes + 255) / 256 * 256;
        BC_REQUIRE(used + bytes <= cap, BC_ERR_ARG, "operation needs more workspace than the fixed scratch holds");
        void *p = base + used;
        used += bytes;
        return p;
    }
};
extern thread_local Arena *tl_arena;
struct ArenaScope {
    Arena a;
    Arena *prev;
    ArenaScope(void *base, size_t cap) : a{(char *)base, cap}, prev(tl_arena) { tl_arena = &a; }
    ~ArenaScope() { tl_arena = prev; }
};

// Device workspace buffer: from the context pool (returned when the last owner
// drops it), or from the thread's arena when one is installed.
struct Buf {
    bc_ctx *c;
    void *p;
    bool pooled;
    Buf(bc_ctx *ctx, size_t bytes)
        : c(ctx), p(tl_arena ? tl_arena->take(bytes) : ctx->pool.alloc(bytes)), pooled(!tl_arena) {}
    ~Buf() {
        if (pooled) c->pool.release(p);
    }
    Buf(const Buf &) = delete;
    Buf &operator=(const Buf &) = delete;
};
using BufP = std::shared_ptr<Buf>;

inline BufP make_buf(bc_ctx *c, size_t bytes) { return std::make_shared<Buf>(c, bytes); }

// A batch of ciphertexts [count][ncomp][level+1][N] in device memory.
struct CtB {
    u64 *data = nullptr;
    int count = 0, level = 0, ncomp = 2;
    double noise = 0;  // estimated noise bits (see NoiseModel)
    BufP own;  // null for caller-owned memory
    size_t ct_words(int N) const { return (size_t)ncomp * (level + 1) * N; }
    CtB slice(int first, int n, int N) const {
        CtB s = *this;
        s.data = data + (size_t)first * ct_words(N);
        s.count = n;
        return s;
    }
};

CtB alloc_ct(bc_ctx *c, int count, int level, int ncomp);
CtB from_abi(const bc_ctx *c, const bc_ctb *x);

void mod_switch(bc_ctx *c, const CtB &in, const CtB &out, hipStream_t st);
// x brought down to out.level, written to out (a copy when the levels agree)
void to_level_into(bc_ctx *c, const CtB &x, const CtB &out, hipStream_t st);
void tensor(bc_ctx *c, const CtB &a, const CtB &b, const CtB &out, hipStream_t st);
void relin(bc_ctx *c, const bc_keys *k, const CtB &in3, const CtB &out, hipStream_t st);
void mul_relin(bc_ctx *c, const bc_keys *k, const CtB &a, const CtB &b, const CtB &out, hipStream_t st);
void mul_relin_add(bc_ctx *c, const bc_keys *k, const CtB &a, const CtB &b, const CtB &add, const CtB &out,
                   hipStream_t st);
CtB mul(bc_ctx *c, const bc_keys *k, const CtB &a, const CtB &b, hipStream_t st);
// Workspace bytes mul_relin takes for `count` products at level lv (each
// buffer rounded up to 256 bytes, none reused within the call).
size_t mul_relin_workspace(const bc_ctx *c, int count, int lv);
void rotate(bc_ctx *c, const bc_keys *k, const CtB &in, int steps, const CtB &out, hipStream_t st);
// out = in + rotate(in) (out != in)
void rotate_add(bc_ctx *c, const bc_keys *k, const CtB &in, int steps, const CtB &out, hipStream_t st);
void add_sub(bc_ctx *c, const CtB &a, const CtB &b, const CtB &out, bool sub, hipStream_t st);
CtB add(bc_ctx *c, const CtB &a, const CtB &b, hipStream_t st);
CtB sub(bc_ctx *c, const CtB &a, const CtB &b, hipStream_t st);
void mul_scalar(bc_ctx *c, const CtB &a, int64_t v, const CtB &out, hipStream_t st);
void add_const(bc_ctx *c, const CtB &a, int64_t v, const CtB &out, hipStream_t st);
void copy_ct(const bc_ctx *c, const CtB &src, const CtB &dst, hipStream_t st);
int64_t centred(const bc_ctx *c, int64_t v);
int out_level_mul(int la, int lb);

// keys and client side
bc_keys *keygen(bc_ctx *c, const int8_t *s, const u64 *words, const int32_t *err, const int32_t *steps, int nrot);
// key sets as a flat coefficient-domain blob (checkpoint / resume, parity)
size_t keys_export(bc_ctx *c, const bc_keys *k, void *buf, size_t cap);
bc_keys *keys_import(bc_ctx *c, const void *buf, size_t size);
void encrypt(bc_ctx *c, const bc_keys *k, const u32 *slots, const int8_t *u, const int32_t *err, const CtB &out,
             hipStream_t st);
void decrypt_poly(bc_ctx *c, const bc_keys *k, const CtB &in, u32 *coeffs, hipStream_t st);
void decode_slots(const bc_ctx *c, const u32 *coeffs, u32 *slots, int count);
// the plaintext polynomial itself (coefficients taken mod p)
void encrypt_poly(bc_ctx *c, const bc_keys *k, const u32 *coeffs, const int8_t *u, const int32_t *err, const CtB &out,
                  hipStream_t st);
// F_{p^d} slots in the power basis: elems[count][M][d] <-> coeffs[count][N]
void encode_fpd(const bc_ctx *c, const u32 *elems, int count, u32 *m);
void decode_fpd(const bc_ctx *c, const u32 *m, int count, u32 *elems);
// rotation steps of the Frobenius powers p^(2^b), b < log2(N/M)
std::vector<int> frobenius_steps(const bc_ctx *c);
// digit k of every slot's F_{p^d} element as F_p slot values: out holds
// ndig * in.count ciphertexts, digit-major, at in.level; rotation keys for
// every Frobenius step
void extract_digits(bc_ctx *c, const bc_keys *k, const CtB &in, const int *digits, int ndig, const CtB &out,
                    hipStream_t st);
void import_ct(bc_ctx *c, const u64 *host, const CtB &out, hipStream_t st);
void export_ct(bc_ctx *c, const CtB &in, u64 *host, hipStream_t st);
u64 galois_for_step(const bc_ctx *c, int step);

// comparison circuits (digit planes, most significant first)
struct CompareResult {
    CtB lt, mx, mn;  // mx, mn: plane-major [ndig * count]
};
// circuit: BC_CIRCUIT_UNIVARIATE (digits in [0, (p-1)/2], the
// Paterson-Stockmeyer schedule) or BC_CIRCUIT_BIVARIATE (digits in [0, p-1])
CompareResult compare(bc_ctx *c, const bc_keys *k, int ndig, const CtB *A, const CtB *B, bool want_mm, hipStream_t st,
                      int circuit = BC_CIRCUIT_UNIVARIATE);
// Slot-packed integers (l digits each in consecutive slots of a row, most
// significant first): LT valid at each integer's first slot.  Needs rotation
// keys for steps 1, 2, ..., l/2.
CtB compare_packed(bc_ctx *c, const bc_keys *k, const CtB &A, const CtB &B, int l, int circuit, hipStream_t st);
// Minimum (want_max: maximum) over every window of `window` consecutive
// slots of a row, at the window's first slot.  Rotation keys 1, 2, ..., window/2.
CtB tournament(bc_ctx *c, const bc_keys *k, const CtB &X, int window, bool want_max, int circuit, hipStream_t st);
// Output level and noise estimate of those two (BC_ERR_LEVEL when too deep).
void packed_levels(const NoiseModel &m, int in_level, double in_noise, int l, int circuit, int *lv, double *nb);
void tournament_levels(const NoiseModel &m, int in_level, double in_noise, int window, int circuit, int *lv,
                       double *nb);
// Levels and noise estimates of the outputs of a comparison of inputs at
// in_level with noise in_noise; BC_ERR_LEVEL when a step of the circuit would
// exceed its level's noise budget (the circuit is deeper than the chain).
struct CircuitNoise {
    int lt_level, mm_level;
    double lt_noise, mm_noise;
};
void compare_levels(const NoiseModel &m, int in_level, double in_noise, int ndig, bool want_mm, CircuitNoise *out,
                    int circuit = BC_CIRCUIT_UNIVARIATE);

}  // namespace bc
