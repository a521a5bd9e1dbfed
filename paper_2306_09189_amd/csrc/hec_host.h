// hec_host.h -- host-side number theory, tables and the slot encoder.
#pragma once
#include <stddef.h>
#include <stdint.h>
#include <vector>

namespace hec {

typedef unsigned __int128 u128;

uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q);
uint64_t powmod(uint64_t a, uint64_t e, uint64_t q);
uint64_t invmod(uint64_t a, uint64_t q);
bool is_prime(uint64_t m);
// first prime 2^bits - j*2n + 1 (j >= 1) not in `taken`; 0 if none above 2^(bits-1)
uint64_t find_prime(uint32_t bits, uint32_t n, const std::vector<uint64_t> &taken);
uint64_t find_root_2n(uint64_t q, uint32_t n);  // element of order 2n
uint64_t shoup_of(uint64_t w, uint64_t q);       // floor(w * 2^64 / q)

// Gaussian cumulative table (sigma, |x| <= 19), 63-bit thresholds, exact unless
// a threshold lies within ~2^-40 of an integer; false for sigma outside [2, 8]
// (below 2 the tail beyond 19 is too small for the ~100-bit evaluation).
bool gauss_table(double sigma, uint64_t T[19]);

// Tables of the slot encoder (the transforms run on the GPU): tw[4e .. 4e+3] =
// cos(pi e / n) and sin(pi e / n) as double-double pairs (hi, lo, hi, lo), e < 2n,
// from a double-double Taylor evaluation; root[j] = (5^j mod 2n - 1) / 2, j < n/2,
// the FFT position of the root zeta^(5^j) that carries slot j.
struct EncoderTables {
    explicit EncoderTables(uint32_t logn);
    std::vector<double> tw;
    std::vector<uint32_t> root;
};

}  // namespace hec
