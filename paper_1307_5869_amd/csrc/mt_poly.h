// Host-side MT19937 jump polynomials (context set-up).  Pure C++: built by
// the host compiler with the x86 carry-less multiply.
#pragma once

#include <cstdint>

namespace prand {

constexpr int kMtDeg = 19937;      // degree of the characteristic polynomial phi
constexpr int kMtPolyWords = 624;  // 32-bit words per reduced polynomial

// Digit tables for block splitting by id * 2^e (e = the block exponent): the
// low 48 bits of an id as kMtLoDigits digits of kMtLoBits bits, the top 16
// bits as two bytes.
constexpr int kMtLoBits = 16;
constexpr int kMtLoDigits = 48 / kMtLoBits;
constexpr int kMtLoSize = 1 << kMtLoBits;

// ladder: nladder polynomials x^(2^b) mod phi, b < nladder (624 words each).
// dig_lo (may be null): kMtLoDigits x kMtLoSize polynomials
// x^(d * 2^(digit_e + kMtLoBits k)) mod phi; dig8hi (may be null): 2 x 256
// polynomials x^(d * 2^(digit_e + 48 + 8 j)) mod phi (d = 0 left zero in
// both).  phi comes from Berlekamp-Massey on MT19937 output bits.  Returns
// false if phi has the wrong degree or the ladder is too short.
bool mt_build_polys(uint32_t* ladder, int nladder, uint32_t* dig_lo, uint32_t* dig8hi, int digit_e);

// Whole-block jumps: blk (nblk polynomials) gets x^(624 * 2^(first + i))
// mod phi, i < nblk (needs first + nblk + 9 <= nladder of the 2^b ladder,
// rebuilt here), and inv gets x^(-1) mod phi = (phi - 1) / x (phi(0) = 1: the
// transition is invertible).  Returns false as mt_build_polys does.
bool mt_build_block_polys(int nladder, int first, int nblk, uint32_t* blk, uint32_t* inv);

}  // namespace prand
