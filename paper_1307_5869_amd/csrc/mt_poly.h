// Host-side MT19937 jump polynomials (context set-up).  Pure C++: built by
// the host compiler with the x86 carry-less multiply.
#pragma once

#include <cstdint>

namespace prand {

constexpr int kMtDeg = 19937;      // degree of the characteristic polynomial phi
constexpr int kMtPolyWords = 624;  // 32-bit words per reduced polynomial

// Digit tables for block splitting by id * 2^e (e = the block exponent): the
// low 48 bits of an id as four 12-bit digits, the top 16 bits as two bytes.
constexpr int kMtDig12Count = 4;

// ladder: nladder polynomials x^(2^b) mod phi, b < nladder (624 words each).
// dig12 (may be null): 4 x 4096 polynomials x^(d * 2^(digit_e + 12 k)) mod phi
// for k < 4, d < 4096; dig8hi (may be null): 2 x 256 polynomials
// x^(d * 2^(digit_e + 48 + 8 j)) mod phi for j < 2, d < 256 (d = 0 left zero
// in both).  phi comes from Berlekamp-Massey on MT19937 output bits.  Returns
// false if phi has the wrong degree or the ladder is too short.
bool mt_build_polys(uint32_t* ladder, int nladder, uint32_t* dig12, uint32_t* dig8hi, int digit_e);

}  // namespace prand
