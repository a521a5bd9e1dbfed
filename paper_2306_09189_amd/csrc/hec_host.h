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

// Gaussian cumulative table (sigma, |x| <= 19), 63-bit thresholds.
void gauss_table(double sigma, uint64_t T[19]);

// Real-slot encoder: m_t = round_half_away(scale * (2/n) sum_j z_j cos(pi (5^j t mod 2n)/n)),
// evaluated through a length-n double-double FFT over the odd powers of zeta.
class Encoder {
public:
    explicit Encoder(uint32_t logn);
    // returns false if a coefficient exceeds 2^62 in magnitude
    bool encode(const double *z, size_t nz, double scale, int64_t *m) const;
    // z_j = (1/scale) sum_t m_t cos(pi (5^j t mod 2n)/n), double precision
    void decode(const double *m, double scale, double *z, size_t nz) const;
    uint32_t n() const { return n_; }

private:
    uint32_t n_;
    std::vector<double> ch_, cl_, sh_, sl_;  // cos/sin(pi e / n), e < 2n, as double-double
    std::vector<uint32_t> slot_root_;        // (5^j mod 2n - 1)/2, j < N
};

}  // namespace hec
