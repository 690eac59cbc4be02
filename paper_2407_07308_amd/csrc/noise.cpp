// noise.cpp -- host-side noise estimates and the budget check behind
// BC_ERR_LEVEL.
//
// BGV decrypts correctly while [c0 + c1 s]_Q, i.e. m + p e, stays below Q/2
// in magnitude; every multiplication roughly squares it and every modulus
// switch divides it by the dropped prime and adds a rounding term (paper,
// Background, "Word-wise Universal FHE Scheme": the modulus chain; HElib
// tracks the same quantity and refuses operations that would exhaust it).
// All figures are log2 of an infinity-norm bound.

#include <cmath>

#include "bc_internal.h"

namespace bc {

namespace {
constexpr double kSigma = 3.2;  // error deviation of the key and encryption randomness
// Every bound below is doubled (one bit) so that the estimate stays above
// the exact noise measured on the oracle's ciphertexts (the estimate without
// it was up to 0.4 bits below on fresh encryptions at N = 2^12).
constexpr double kSafety = 2.0;

double lg(double x) { return std::log2(x); }
// log2 (2^a + 2^b)
double lsum(double a, double b) {
    if (a < b) std::swap(a, b);
    if (std::isinf(b)) return a;
    return a + std::log2(1.0 + std::exp2(b - a));
}
}  // namespace

NoiseModel::NoiseModel(const bc_params &prm, const std::vector<u64> &mod) {
    N = 1 << prm.logN;
    nQ = prm.nQ;
    nP = prm.nP;
    dnum = prm.dnum;
    alpha = (prm.nQ + prm.dnum - 1) / prm.dnum;
    p = (double)prm.p;
    z = std::sqrt(2.0 * std::log(2.0 * N));
    double acc = 0;
    for (int i = 0; i < nQ; i++) {
        lq.push_back(lg((double)mod[i]));
        acc += lq.back();
        lQ.push_back(acc);
    }
    for (int j = 0; j < nP; j++) lP += lg((double)mod[nQ + j]);
}

// p (e u + e0 + e1 s) + m: e u and e1 s have coefficients of deviation
// sigma sqrt(2N/3) (ternary u, s), e0 of sigma; |m| <= p/2 (centred).
double NoiseModel::fresh() const { return lg(kSafety * (p * kSigma * z * std::sqrt(4.0 * N / 3.0 + 1.0) + p / 2)); }

double NoiseModel::add(double a, double b) const { return lsum(a, b); }

double NoiseModel::scalar(double a, double absc) const { return a + lg(std::max(1.0, absc)); }

double NoiseModel::add_const(double a) const { return lsum(a, lg(p / 2)); }

// Tensor: a coefficient of the product of two noise polynomials sums N
// products, so its deviation is sqrt(N) times the product of theirs; bounds
// of z deviations give sqrt(N) Ba Bb / z.  Key switching adds
// p sum_j d_j e_j / P (digits below alpha Q_j after raising, Q_j < 2^(alpha
// bits)) and the rounding of the exact division by P, p (r0 + r1 s) with
// |r| <= (nP + 1) / 2.
double NoiseModel::tensor(double a, double b) const { return a + b + 0.5 * lg((double)N) - lg(z); }

double NoiseModel::product(int level, double a, double b, double c) const {
    return key_switch(level, lsum(tensor(a, b), c));
}

double NoiseModel::key_switch(int level, double t) const {
    const int nact = level / alpha + 1;
    double lqd = 0;  // log2 of the largest digit modulus at this level
    for (int j = 0; j < nact; j++) {
        double d = 0;
        for (int i = j * alpha; i < std::min((j + 1) * alpha, level + 1); i++) d += lq[i];
        lqd = std::max(lqd, d);
    }
    const double ks = lg(kSafety * p * kSigma * z * std::sqrt((double)N * nact) * alpha) + lqd - lP;
    const double md = lg(kSafety * p * 0.5 * (nP + 1) * (1.0 + z * std::sqrt(2.0 * N / 3.0)));
    return lsum(lsum(t, ks), md);
}

// (c - p t) / q_l with |t| <= q_l / 2: the noise divided by q_l plus
// p (tau0 + tau1 s), tau uniform in [-1/2, 1/2] (deviation of tau1 s:
// sqrt(2N/3) / sqrt(12)).
double NoiseModel::mod_switch(int level, double a) const {
    return lsum(a - lq[level], lg(kSafety * p * (0.5 + z * std::sqrt(N / 18.0))));
}

// the automorphism permutes the coefficients (with signs): the norm stays
double NoiseModel::rotate(int level, double a) const { return key_switch(level, a); }

void NoiseModel::require(int level, double bits, const char *what) const {
    if (!(bits <= budget(level))) {
        char buf[200];
        std::snprintf(buf, sizeof buf, "%s: estimated noise 2^%.1f exceeds the budget 2^%.1f at level %d", what,
                      bits, budget(level), level);
        throw Error(BC_ERR_LEVEL, buf);
    }
}

}  // namespace bc
