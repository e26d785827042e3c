// Host-side MT19937 jump polynomials (context set-up).  Pure C++: built by
// the host compiler with the x86 carry-less multiply.
#pragma once

#include <cstdint>

namespace prand {

constexpr int kMtDeg = 19937;      // degree of the characteristic polynomial phi
constexpr int kMtPolyWords = 624;  // 32-bit words per reduced polynomial

// ladder: nladder polynomials x^(2^b) mod phi, b < nladder (624 words each).
// digits (may be null): 8 x 256 polynomials x^(d * 2^(digit_e + 8 j)) mod phi
// for byte position j < 8 and d < 256 (d = 0 left zero).  phi comes from
// Berlekamp-Massey on MT19937 output bits.  Returns false if phi has the
// wrong degree.
bool mt_build_polys(uint32_t* ladder, int nladder, uint32_t* digits, int digit_e);

}  // namespace prand
