// bluestein.h -- transforms of the non-power-of-two cyclotomic rings
// Z_q[X]/(Phi_m(X)), m odd: coefficients <-> values at the primitive m-th
// roots of unity, by Bluestein's method on the library's power-of-two
// transforms (paper, Background, "Efficient Polynomial and NTT": the
// BluesteinNTT; The Design of BoostCom, "GPU-related Optimizations": the
// branch-free polynomial filter with its offline prefix sum).
#pragma once

#include "bc_internal.h"

struct bc_bluestein;

namespace bc {

bc_bluestein *bluestein_create(int m, int nprimes, int bits);
void bluestein_destroy(bc_bluestein *b);
// degree phi(m), convolution length, primes (nprimes words)
void bluestein_info(const bc_bluestein *b, int *n, int *conv_len, u64 *moduli);
// in/out: [count][nprimes][n] canonical words, device memory, on `st`
void bluestein_forward(bc_bluestein *b, const u64 *in, u64 *out, int count, hipStream_t st);
void bluestein_inverse(bc_bluestein *b, const u64 *in, u64 *out, int count, hipStream_t st);

}  // namespace bc
