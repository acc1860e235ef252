// gf2_modulus.h -- the library's modulus convention (see gf2_modulus.cpp).
#pragma once
#include <stdint.h>

#include <vector>

namespace qext {

// Largest degree searched at run time when the built-in table (every
// multiple of 8 up to 8192, and 16384) lacks it; a search takes about a
// second at 10000 bits and minutes at 32768 on 8 host threads.
constexpr uint32_t kSearchLimit = 32768;

// Rabin's test for P = t^m + sum t^taps[k] + 1.
bool modulus_is_irreducible(uint32_t m, const uint32_t* taps, uint32_t n_taps);

// Search for the conventional modulus of degree m (no table, no cache):
// *taps receives the non-leading nonzero exponents in decreasing order.
bool search_modulus(uint32_t m, std::vector<uint32_t>* taps);

// Conventional modulus: built-in table, else a cached search up to
// kSearchLimit.
bool default_modulus(uint32_t m, std::vector<uint32_t>* taps);

}  // namespace qext
