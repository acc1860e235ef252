// ext_params.cpp -- host-side parameter rule and security bounds of the
// block-wise extractors (no GPU work).
//
//   * Algorithm 1's parameters: n_e = ceil(24 / (2 delta - 1)) elements per
//     block and q = b * ceil(log2(N / (eps n_e)) / b) bits per element.
//   * Theorem 3.3: one block's output is within
//     sqrt(3) * 2^(-1/4 - (delta/4 - 1/8) q n_e + 2q) of uniform.
//   * Theorem 3.6: Algorithm 2's first k outputs (q_l = q_1 + (l-1) Delta b)
//     are within the sum of those per-block bounds, and for Delta > 0 below
//     sqrt(3) 2^(-1/4 - q_1) / (1 - 2^(-Delta b)); they hold
//     m_k = k q_1 + k (k-1) Delta b / 2 bits.
//
// The per-block exponents of Algorithm 2 form an arithmetic progression, so
// the sum over k blocks is a geometric series, evaluated here in closed form
// in the log domain (no loop over k).
#include <math.h>
#include <stdint.h>

#include "../../include/qrng_ext.h"

namespace {

constexpr double kLog2Sqrt3 = 0.79248125036057812;  // log2(3) / 2

// log2(1 - 2^x) for x < 0, accurate when 2^x is close to 1 (expm1) and when
// it is close to 0 (log1p)
double log2_one_minus_exp2(double x) {
    if (x > -1.0) return log2(-expm1(x * M_LN2));
    return log1p(-exp2(x)) / M_LN2;
}

// Exponent of Theorem 3.3's bound, without the sqrt(3) factor.
double block_exponent(double n_e, double q, double delta) {
    return -0.25 - (delta / 4.0 - 0.125) * q * n_e + 2.0 * q;
}

}  // namespace

extern "C" {

int ext_choose_params(uint32_t sample_bits, uint64_t delta_num, uint64_t delta_den,
                      double log2_n_samples, double log2_eps, uint32_t* n_e, uint32_t* q) {
    if (!n_e || !q || sample_bits == 0 || delta_den == 0) return EXT_EINVAL;
    // 1/2 < delta = num/den <= 1
    const unsigned __int128 num = delta_num, den = delta_den;
    if (2 * num <= den || num > den) return EXT_EINVAL;
    if (!(log2_eps < 0.0) || !isfinite(log2_eps) || !isfinite(log2_n_samples))
        return EXT_EINVAL;
    const unsigned __int128 step = 2 * num - den;  // (2 delta - 1) * den
    const unsigned __int128 ne = (24 * den + step - 1) / step;
    if (ne > 0xffffffffu) return EXT_EINVAL;
    const double t = (log2_n_samples - log2_eps - log2((double)ne)) / (double)sample_bits;
    if (!(t > 0.0) || t > 1e9) return EXT_EINVAL;
    const double k = ceil(t);
    const double qq = k * (double)sample_bits;
    if (qq > 2147483647.0) return EXT_EINVAL;
    *n_e = (uint32_t)ne;
    *q = (uint32_t)qq;
    return EXT_OK;
}

double ext_block_error_log2(uint32_t n_e, uint32_t q, double delta) {
    if (n_e == 0 || q == 0 || !(delta > 0.0 && delta <= 1.0)) return NAN;
    return kLog2Sqrt3 + block_exponent(n_e, q, delta);
}

int ext_stream_error_log2(uint32_t n_e, uint32_t q1, uint32_t delta_steps, uint32_t sample_bits,
                          double delta, uint64_t k, double* log2_sum, double* log2_closed) {
    if (n_e == 0 || q1 == 0 || sample_bits == 0 || k == 0 || !(delta > 0.0 && delta <= 1.0))
        return EXT_EINVAL;
    const double e1 = block_exponent(n_e, q1, delta);
    // exponent change from one block to the next
    const double r = (double)delta_steps * sample_bits * (2.0 - (delta / 4.0 - 0.125) * n_e);
    const double kd = (double)k;
    double s;
    if (r == 0.0) {
        s = e1 + log2(kd);
    } else if (r < 0.0) {
        // 2^e1 (1 - 2^(k r)) / (1 - 2^r)
        s = e1 + log2_one_minus_exp2(kd * r) - log2_one_minus_exp2(r);
    } else {
        // largest term last: 2^(e1 + (k-1) r) (1 - 2^(-k r)) / (1 - 2^(-r))
        s = e1 + (kd - 1.0) * r + log2_one_minus_exp2(-kd * r) - log2_one_minus_exp2(-r);
    }
    if (log2_sum) *log2_sum = kLog2Sqrt3 + s;
    if (log2_closed)
        *log2_closed = delta_steps == 0
                           ? INFINITY
                           : kLog2Sqrt3 - 0.25 - (double)q1 -
                                 log2_one_minus_exp2(-(double)delta_steps * sample_bits);
    return EXT_OK;
}

int ext_output_bits(uint32_t q1, uint32_t delta_steps, uint32_t sample_bits, uint64_t k,
                    uint64_t* m_k) {
    if (!m_k) return EXT_EINVAL;
    // beyond 2^33 blocks the growth term alone exceeds 64 bits
    if (delta_steps && k > (1ull << 33)) return EXT_EINVAL;
    const unsigned __int128 kk = k;
    const unsigned __int128 m =
        kk * q1 + (kk * (kk - (k ? 1 : 0)) / 2) * ((unsigned __int128)delta_steps * sample_bits);
    if (m > (unsigned __int128)UINT64_MAX) return EXT_EINVAL;
    *m_k = (uint64_t)m;
    return EXT_OK;
}

}  // extern "C"
