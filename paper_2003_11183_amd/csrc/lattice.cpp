// Host side of the lattice: Richtmyer generators and the random shifts.
//
// Generator c is A_c = floor(frac(sqrt(p_{c+1})) 2^64) for the consecutive
// primes p_1 = 2, p_2 = 3, ... (Richtmyer's rule, named in Section 2.1 of
// the paper).  It is found exactly: with q = floor(sqrt(p)), A_c is the
// largest F < 2^64 with (q 2^64 + F)^2 <= p 2^128, decided bit by bit in
// 192-bit arithmetic.  The shifts are SplitMix64 outputs (Steele, Lea and
// Flood 2014): output i of state s is mix(s + (i + 1) gamma).
#include <cmath>
#include <cstdint>
#include <vector>

#include "internal.hpp"

namespace tlrqmc {

namespace {

using u128 = unsigned __int128;

std::vector<uint32_t> first_primes(int64_t count) {
  std::vector<uint32_t> out;
  if (count <= 0) return out;
  double est = static_cast<double>(count) * (std::log(count + 1.0) + std::log(std::log(count + 2.0)) + 3.0);
  int64_t lim = std::max<int64_t>(32, static_cast<int64_t>(est));
  for (;;) {
    std::vector<uint8_t> comp(lim + 1, 0);
    out.clear();
    for (int64_t i = 2; i <= lim; ++i) {
      if (comp[i]) continue;
      out.push_back(static_cast<uint32_t>(i));
      if (static_cast<int64_t>(out.size()) == count) return out;
      for (int64_t j = i * i; j <= lim; j += i) comp[j] = 1;
    }
    lim *= 2;
  }
}

// Is (q 2^64 + F)^2 <= p 2^128 ?  Both sides as 192-bit numbers in three
// 64-bit limbs (lo, mid, hi).
bool square_fits(uint64_t q, uint64_t F, uint64_t p) {
  // (q 2^64 + F)^2 = q^2 2^128 + 2 q F 2^64 + F^2
  const u128 ff = static_cast<u128>(F) * F;
  const u128 qf2 = static_cast<u128>(q) * F * 2u;  // q < 2^11, so this fits
  uint64_t lo = static_cast<uint64_t>(ff);
  u128 mid = (ff >> 64) + static_cast<uint64_t>(qf2);
  u128 hi = (qf2 >> 64) + static_cast<u128>(q) * q + (mid >> 64);
  // right side: p 2^128 -> limbs (0, 0, p)
  (void)lo;
  if (hi != p) return hi < p;
  return static_cast<uint64_t>(mid) == 0 && lo == 0;
}

}  // namespace

std::vector<uint64_t> richtmyer_generators(int64_t dim) {
  const std::vector<uint32_t> ps = first_primes(dim);
  std::vector<uint64_t> A(dim);
  for (int64_t c = 0; c < dim; ++c) {
    const uint64_t p = ps[c];
    uint64_t q = static_cast<uint64_t>(std::sqrt(static_cast<double>(p)));
    while (q * q > p) --q;
    while ((q + 1) * (q + 1) <= p) ++q;
    uint64_t F = 0;
    for (int bit = 63; bit >= 0; --bit) {
      const uint64_t cand = F | (uint64_t{1} << bit);
      if (square_fits(q, cand, p)) F = cand;
    }
    A[c] = F;
  }
  return A;
}

std::vector<uint64_t> splitmix64_table(uint64_t seed, int64_t count) {
  std::vector<uint64_t> out(count);
  uint64_t s = seed;
  for (int64_t i = 0; i < count; ++i) {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    out[i] = z ^ (z >> 31);
  }
  return out;
}

}  // namespace tlrqmc
