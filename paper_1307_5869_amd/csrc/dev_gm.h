// GM19, GM29, GM31, GM55, GM61, GQ58.1, GQ58.3, GQ58.4 on gfx950: ensembles of
// s torus maps x_i^(n) = k x_i^(n-1) - q x_i^(n-2) mod g (paper, equation
// rec1; k, q, g, v of Table 2).  Each element contributes a v-bit digit
// floor(2^v x / g) per step; digits are packed element 0 first, most
// significant bit first, into 32-bit words (GQ58.3: 36 bits per step, 9 words
// per 8 steps).
//
// This header holds the per-generator arithmetic, the jumps, and the v = 1
// ensembles' (s = 32) wavefront routine: one lane per element, half a
// wavefront per stream, one ballot per step packs a word.  The v >= 3
// ensembles (GM55, GQ58.3, GQ58.4) run one lane per section (dev_gmlane.h).
//
// Arithmetic is exact: special-form reductions (2^19-1, 2^29-3, 2^61-1,
// 2^51-129) in integers.  For g = p 2^t (GM55: t = 4, GQ58: t = 29) the even
// k and q kill the 2-adic part within n0 steps; from then on x = 2^t y with y
// following the same recurrence mod p and the digit equal to
// floor(2^v y / p), so the kernels run exact mod-g steps only until every
// element of the wavefront has collapsed and then switch to the mod-p
// recurrence.  In the steady state an element is held as a redundant
// residue (congruent to the exact value, possibly shifted by a constant, in
// a range a little wider than the modulus), so no step needs a final
// conditional subtraction; digits are read off that form and states are
// written back exact.
// GM/GQ device code shared by the GM/GQ kernels and the batched kernel.
#pragma once

#include <type_traits>

#include "prand_impl.h"

namespace prand {
namespace gm {

typedef unsigned __int128 u128;

// An empty asm that the optimiser cannot see through: the value is taken as
// computed, so a constant folded into it is not re-associated into a later
// sum (which would cost an extra add instead of a multiply-add's addend).
template <class T>
__device__ __forceinline__ T pin(T v) {
  asm("" : "+v"(v));
  return v;
}

// ------------------------------------------------------------ per generator
template <int G>
struct Eng;

// GM29, GM31, GM61 and GQ58.1 keep each element in a redundant range
// [0, g + d) (GM29 and GQ58.1: shifted by a constant c, the stored value
// congruent to x + c), so no step pays for a final conditional subtraction;
// the digit is read off the redundant value with two compares, and from_fast
// returns the exact value.  The bounds below hold for every input in the
// range.  GM19 (g < 2^20) keeps a centred residue in FP32 instead.

// GM19: g = 2^19 - 1, k = 15, q = 28.  Each element is held as its centred
// residue r in [-(g - 1) / 2, (g - 1) / 2], an integer-valued float, and a
// step is exact FP32 arithmetic (one multiply and three FMAs, all issued at
// gfx950's fast rate, where the 24-bit integer multiply-adds issue at the
// slow one):
//  * t = 15 zc - 28 zp: |t| <= 43 (g - 1) / 2 < 2^24, so the product 28 zp
//    and the FMA sum are exact;
//  * k = rint(t / g) from one FMA with the rounding constant 1.5 2^23: 1/g
//    rounded to FP32 is 2^-19 (1 + 2^-19), within 2^-38 relative of 1/g, so
//    t/g is evaluated within 2^-33, while t/g (g odd) is never closer than
//    1/(2g) > 2^-20 to a half-integer: k is the exact nearest integer;
//  * r = t - k g is exact (k g < 2^24) and lies in the centred range again.
// The digit floor(2 x / g) of x = r mod g (x = r, or r + g for r < 0) is 1
// exactly when r < 0.
template <>
struct Eng<0> {
  static constexpr bool kComposite = false;
  using F = float;
  static constexpr uint32_t g = 524287u;
  static constexpr float kInvG = 1.0f / 524287.0f;   // RN(1/g) = 2^-19 (1 + 2^-19)
  static constexpr float kRound = 12582912.0f;       // 1.5 2^23: FMA result rounded to an integer
  __device__ static F to_fast(uint64_t x) { return (float)((int)x - (x > (g - 1) / 2 ? (int)g : 0)); }
  __device__ static uint64_t from_fast(F z) {
    const int r = (int)z;
    return (uint64_t)(r < 0 ? r + (int)g : r);
  }
  __device__ static F step(F zc, F zp) {
    const float t = __builtin_fmaf(15.0f, zc, -28.0f * zp);
    const float k = __builtin_fmaf(t, kInvG, kRound) - kRound;
    return __builtin_fmaf(-k, (float)g, t);
  }
  __device__ static bool digit(F z) { return z < 0.0f; }
};

// GM29: g = 2^29 - 3, k = 4, q = 2; z in [0, g + 19], z = x - 38 (mod g).
// a = 2 zc + (g + 19) - zp < 3 g + 58 < 2^31 and 2 a = 3 floor(a / 2^28) +
// 2 (a mod 2^28) (mod g) <= g + 16; the constant g + 19 adds 38 = -2 c
template <>
struct Eng<1> {
  static constexpr bool kComposite = false;
  using F = uint32_t;
  static constexpr uint32_t g = 536870909u;
  __device__ static F to_fast(uint64_t x) { return x >= 38u ? (F)x - 38u : (F)x + (g - 38u); }
  __device__ static uint64_t from_fast(F z) { return z + 38u < g ? z + 38u : z + 38u - g; }
  __device__ static F step(F zc, F zp) {
    const uint32_t a = 2u * zc + pin((g + 19u) - zp);
    return ((a & 0x0FFFFFFFu) << 1) + __umul24(3u, a >> 28);
  }
  // x >= (g + 1) / 2 with x = z + 38 (mod g)
  __device__ static bool digit(F z) { return (z >= (g + 1) / 2 - 38u) & (z < g - 38u); }
};

// GM31: g = 2^31 - 1, k = 11, q = 14; z in [0, g + 39].
// t = 11 zc + 14 (2 g - zp) < 39 g + 430, folded with 2^31 = 1 (mod g) to at
// most g + 38
template <>
struct Eng<2> {
  static constexpr bool kComposite = false;
  using F = uint32_t;
  static constexpr uint32_t g = 2147483647u;
  __device__ static F to_fast(uint64_t x) { return (F)x; }
  __device__ static uint64_t from_fast(F z) { return z >= g ? z - g : z; }
  __device__ static F step(F zc, F zp) {
    const uint64_t t = (uint64_t)11u * zc + (uint64_t)14u * (2u * g - zp);
    return ((uint32_t)t & g) + (uint32_t)(t >> 31);
  }
  __device__ static bool digit(F z) { return (z >= (1u << 30)) & (z < g); }
};

// GM61: g = 2^61 - 1, k = 24, q = 74; z in [0, 2^61 + 98 2^32).
// 24 zc + 74 s with s = 2 g - zp < 2^62, in 32-bit halves: B = 24 zc_hi +
// 74 s_hi < 2^37 and B 2^32 = floor(B / 2^29) + (B mod 2^29) 2^32 (mod g);
// A = 24 zc_lo + 74 s_lo + floor(B / 2^29) < 98 2^32 + 196, and the result
// A + (B mod 2^29) 2^32 only adds to the high word
template <>
struct Eng<4> {
  static constexpr bool kComposite = false;
  using F = uint64_t;
  static constexpr uint64_t g = 2305843009213693951ull;
  __device__ static F to_fast(uint64_t x) { return x; }
  __device__ static uint64_t from_fast(F z) { return z >= g ? z - g : z; }
  __device__ static F step(F zc, F zp) {
    const uint64_t s = 2 * g - zp;
    const uint64_t B = (uint64_t)(uint32_t)(zc >> 32) * 24u + (uint64_t)(uint32_t)(s >> 32) * 74u;
    const uint32_t bhi = __builtin_amdgcn_alignbit((uint32_t)(B >> 32), (uint32_t)B, 29);
    const uint64_t A = (uint64_t)(uint32_t)zc * 24u + pin((uint64_t)(uint32_t)s * 74u + bhi);
    const uint32_t hi = pin((uint32_t)(A >> 32)) + ((uint32_t)B & 0x1FFFFFFFu);
    return ((uint64_t)hi << 32) | (uint32_t)A;
  }
  __device__ static bool digit(F z) { return ((uint32_t)(z >> 32) >= (1u << 28)) & (z < g); }
};

// GM55: g = 2^4 p, p = 2^51 - 129, k = 256, q = 176, v = 4.  After the
// collapse the kernels keep y = x / 16 (mod p) in [0, p + 78560]:
// s = (zc << 8) + 176 (2p - zp) < 609 p < 2^61 folded once with 2^51 = 129
// (mod p) is at most p + 78431
template <>
struct Eng<3> {
  static constexpr bool kComposite = true;
  static constexpr int t = 4, v = 4;
  static constexpr uint64_t p = 2251799813685119ull;
  static constexpr uint64_t g = p << 4;
  using F = uint64_t;
  __device__ static uint64_t modp_fold(uint64_t h) {   // h < 2^60
    h = (h & ((1ull << 51) - 1)) + 129ull * (h >> 51);
    return h >= p ? h - p : h;
  }
  __device__ static bool collapsed(uint64_t x) { return (x & 15u) == 0; }
  __device__ static uint64_t slow_step(uint64_t xc, uint64_t xp) {
    const uint64_t s = (xc << 8) + 176ull * (g - xp);   // < 2^64
    return (modp_fold(s >> 4) << 4) | (s & 15u);
  }
  __device__ static uint32_t slow_digit(uint64_t x) {  // floor(16 x / 16 p) = floor(x / p)
    const uint64_t d0 = x >> 51;
    return (uint32_t)(d0 + ((d0 + 1) * p <= x));
  }
  __device__ static F to_fast(uint64_t x) { return x >> 4; }
  __device__ static uint64_t from_fast(F z) { return (z >= p ? z - p : z) << 4; }
  __device__ static F step(F zc, F zp) {
    const uint64_t s = (zc << 8) + 176ull * (2 * p - zp);
    return (s & ((1ull << 51) - 1)) + 129ull * (s >> 51);
  }
  // floor(16 y / p); a value z in [p, p + 78560] stands for z - p < p / 16
  // (digit 0) and gives 16 here, which the 4-bit mask drops
  __device__ static uint32_t digit(F z) {
    const uint64_t num = z << 4, d0 = num >> 51;
    return (uint32_t)(d0 + ((d0 + 1) * p <= num)) & 15u;
  }
};

// GQ58.x: g = 2^29 p, p = 2^29 - 3, k = 8, q = 48, v = 1, 3, 4
template <int V>
struct EngGQ {
  static constexpr bool kComposite = true;
  static constexpr int t = 29, v = V;
  static constexpr uint64_t p = 536870909ull;
  static constexpr uint64_t g = p << 29;
  __device__ static bool collapsed(uint64_t x) { return (x & 0x1FFFFFFFull) == 0; }
  __device__ static uint64_t slow_step(uint64_t xc, uint64_t xp) {
    const uint64_t s = (xc << 3) + 48ull * (g - xp);   // < 2^64
    uint64_t h = s >> 29;                               // < 2^35
    h = (h & 0x1FFFFFFFull) + 3ull * (h >> 29);
    h = h >= p ? h - p : h;
    return (h << 29) | (s & 0x1FFFFFFFull);
  }
  __device__ static uint32_t slow_digit(uint64_t x) {  // floor(((2^v x) >> 29) / p)
    const uint64_t num = (x << V) >> 29, d0 = num >> 29;
    return (uint32_t)(d0 + ((d0 + 1) * p <= num));
  }
  // fast recurrence on y = x / 2^29 mod p, stored as z = y - 37 (mod p) in
  // [0, p + 166]: u = zc + 6 ((p + 11184779) - zp) < 2^32 (41 * 37 + 48 *
  // 11184779 = p makes the constant cancel the offset) and 8 u = 3 floor(u /
  // 2^26) + 8 (u mod 2^26) (mod p) is at most p + 163
  using F = uint32_t;
  static constexpr uint32_t kP = 536870909u, kM = 0x1FFFFFFFu;
  static constexpr uint32_t kD = 37u, kE = 11184779u;
  __device__ static F to_fast(uint64_t x) {
    const uint32_t y = (uint32_t)(x >> 29);
    return y >= kD ? y - kD : y + (kP - kD);
  }
  __device__ static uint64_t from_fast(F z) { return ((uint64_t)(z + kD >= kP ? z + kD - kP : z + kD)) << 29; }
  __device__ static F step(F zc, F zp) {
    const uint32_t u = zc + 6u * pin((kP + kE) - zp);
    return ((u << 3) & kM) + __umul24(3u, u >> 26);
  }
  // floor(2^v y / p) with y = z + 37: with d0 = floor(2^v y / 2^29),
  // 2^v y - d0 p < 2 p, so the digit is floor((2^v y + 3 d0 + 3) / 2^29) =
  // floor((y + floor((3 d0 + 3) / 2^v)) / 2^(29-v)); d0 may be taken from z
  // instead of y (checked for every z in the range).  z + 37 in [p, p + 203]
  // stands for a value below p / 2^v (digit 0) and gives 2^v, which the
  // v-bit field drops.
  __device__ static uint32_t digit(F z) {
    const uint32_t d0 = z >> (29 - V);
    return ((z + ((__umul24(3u, d0) + (3u + (kD << V))) >> V)) >> (29 - V)) & ((1u << V) - 1u);
  }
};

// GQ58.1 after the collapse: z in [0, p + 184], z = y + 240 (mod p).
// u = zc + 6 ((p + 205) - zp) < 7 p + 1415 < 2^32 and 8 u = 3 floor(u / 2^26)
// + 8 (u mod 2^26) (mod p) <= p + 160; the constant p + 205 = p + 41 * 5
// adds 48 * 205 = 41 * 240 = 41 c
template <>
struct Eng<5> : EngGQ<1> {
  static constexpr uint32_t kC = 240u;
  __device__ static F to_fast(uint64_t x) {
    const uint32_t z = (uint32_t)(x >> 29) + kC;
    return z >= kP ? z - kP : z;
  }
  __device__ static uint64_t from_fast(F z) { return ((uint64_t)(z >= kC ? z - kC : z + (kP - kC))) << 29; }
  __device__ static F step(F zc, F zp) {
    const uint32_t u = zc + 6u * pin((kP + 205u) - zp);
    return ((u << 3) & kM) + __umul24(3u, u >> 26);
  }
  // y >= (p + 1) / 2 with y = z - 240: z < 240 wraps to a large value and
  // stands for y = z - 240 + p >= (p + 1) / 2
  __device__ static bool digit(F z) { return z - kC >= 268435455u; }
};
template <> struct Eng<6> : EngGQ<3> {};
template <> struct Eng<7> : EngGQ<4> {};

// Per-element runner: slow exact-mod-g steps until the whole wavefront has
// collapsed (composite moduli), then the fast recurrence.  The mode only
// switches between steps and is wavefront-uniform.
template <int G>
struct Elem {
  using E = Eng<G>;
  typename E::F fc, fp;   // fast representation
  uint64_t sc, sp;        // exact mod-g values (slow mode)
  bool fast;
  __device__ void load(uint64_t xc, uint64_t xp) {
    if constexpr (E::kComposite) {
      sc = xc; sp = xp; fast = false;
    } else {
      fc = E::to_fast(xc); fp = E::to_fast(xp); fast = true;
    }
  }
  __device__ void maybe_switch() {
    if constexpr (E::kComposite) {
      if (!fast) {
        const bool mine = E::collapsed(sc) && E::collapsed(sp);
        if (__all(mine)) {
          fc = E::to_fast(sc); fp = E::to_fast(sp); fast = true;
        }
      }
    }
  }
  __device__ bool is_fast() const {
    if constexpr (E::kComposite) return fast;
    else return true;
  }
  __device__ uint32_t step_fast() {
    const typename E::F nx = E::step(fc, fp);
    fp = fc; fc = nx;
    return E::digit(nx);
  }
  __device__ uint32_t step_slow() {
    if constexpr (E::kComposite) {
      const uint64_t nx = E::slow_step(sc, sp);
      sp = sc; sc = nx;
      return E::slow_digit(nx);
    } else {
      return step_fast();
    }
  }
  __device__ uint32_t step() { return is_fast() ? step_fast() : step_slow(); }
  // Run body(step) for a block of steps with the mode fixed for the whole
  // block: the switch is taken at the block start, which is exact because a
  // collapsed pair stays collapsed.  Steady state runs the fast body only.
  template <class Body>
  __device__ __forceinline__ void block(Body&& body) {
    maybe_switch();
    if (is_fast()) {
      body([this]() { return step_fast(); });
    } else {
      if constexpr (E::kComposite) body([this]() { return step_slow(); });
    }
  }
  __device__ void get(uint64_t& xc, uint64_t& xp) const {
    if (fast) { xc = E::from_fast(fc); xp = E::from_fast(fp); }
    else { xc = sc; xp = sp; }
  }
};

template <int DT>
__device__ __forceinline__ void put(void* out, uint64_t i, uint32_t w) {
  if (DT == PRAND_U32) ((uint32_t*)out)[i] = w;
  else if (DT == PRAND_F32) ((float*)out)[i] = (float)(w >> 8) * 0x1p-24f;
  else ((double*)out)[i] = (double)w * 0x1p-32;
}

// Lanes L and L + 32 of v take the two halves of a wavefront ballot, with
// v_writelane_b32 and constant lane indices (an inline constant keeps each
// instruction within gfx9's single scalar operand).  The ballot's SGPRs are
// usually written by the VALU compare just before; gfx950 needs two wait
// states between a VALU SGPR write and a VALU read of it, and the compiler
// inserts none for inline assembly, hence the s_nop.
template <int L>
__device__ __forceinline__ uint32_t writelane_pair(uint32_t v, uint32_t lo, uint32_t hi) {
  asm("s_nop 1\n\tv_writelane_b32 %0, %1, %3\n\tv_writelane_b32 %0, %2, %4"
      : "+v"(v)
      : "s"(lo), "s"(hi), "i"(L), "i"(L + 32));
  return v;
}
template <int U, int END, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (U < END) {
    f(std::integral_constant<int, U>{});
    static_for<U + 1, END>(f);
  }
}

// -------------------------------------------------------------- jumping
template <int G>
__device__ __forceinline__ uint64_t fold_special(u128 x, int e, uint64_t c, uint64_t p) {
  const uint64_t mask = (1ull << e) - 1;
  for (int i = 0; i < 3; i++) x = (x & mask) + (u128)c * (uint64_t)(x >> e);
  uint64_t r = (uint64_t)x;
  r = r >= p ? r - p : r;
  r = r >= p ? r - p : r;
  return r;
}
// m0 a + m1 b mod p = 2^e - c with every operand below p: below 2^32
// (GM19, GM29, GM31, GQ58) the products and their sum fit 64 bits, so the
// folds run in 64-bit arithmetic; GM55 and GM61 need 128 bits
template <int G>
__device__ __forceinline__ uint64_t mulsum_mod(uint64_t m0, uint64_t a, uint64_t m1, uint64_t b, int e,
                                               uint64_t c, uint64_t p) {
  if constexpr (G == 3 || G == 4) {
    return fold_special<G>((u128)m0 * a + (u128)m1 * b, e, c, p);
  } else {
    const uint64_t mask = (1ull << e) - 1;
    uint64_t x = m0 * a + m1 * b;   // < 2^63
    for (int i = 0; i < 3; i++) x = (x & mask) + c * (x >> e);
    x = x >= p ? x - p : x;
    return x >= p ? x - p : x;
  }
}
// prime part p = 2^e - c of each generator's modulus
__device__ __forceinline__ void prime_form(int G, int& e, uint64_t& c) {
  switch (G) {
    case 0: e = 19; c = 1; break;
    case 1: e = 29; c = 3; break;
    case 2: e = 31; c = 1; break;
    case 3: e = 51; c = 129; break;
    case 4: e = 61; c = 1; break;
    default: e = 29; c = 3; break;
  }
}

// Jump one element (xc, xp) = (x^(n), x^(n-1)) ahead by N ensemble steps
// (little-endian limbs, N[kMaxLimbs] must be 0 on entry to the ladder part):
// one ladder matrix M^(2^b) mod p per set bit b.  Composite moduli first
// collapse (n0 exact steps) unless the element already has, then jump x/2^t
// mod p; distances below n0 are taken as exact steps.
template <int G>
__device__ __forceinline__ void jump_steps_elem(uint64_t& xc, uint64_t& xp, uint64_t* N,
                                                const uint64_t* __restrict__ ladder) {
  using E = Eng<G>;
  int pe;
  uint64_t pc;
  prime_form(G, pe, pc);
  const uint64_t p = kGmParams[G].p;
  const uint64_t* L = ladder + (size_t)G * kLadder * 4;
  if constexpr (E::kComposite) {
    bool small = true;
    for (int l = 1; l <= kMaxLimbs; l++) small = small && N[l] == 0;
    const uint64_t n0 = (uint64_t)kGmParams[G].n0;
    if (small && N[0] < n0) {
      for (uint64_t i = 0; i < N[0]; i++) { const uint64_t nx = E::slow_step(xc, xp); xp = xc; xc = nx; }
      return;
    }
    if (!(E::collapsed(xc) && E::collapsed(xp))) {
      for (uint64_t i = 0; i < n0; i++) { const uint64_t nx = E::slow_step(xc, xp); xp = xc; xc = nx; }
      uint64_t borrow = n0;
      for (int l = 0; l <= kMaxLimbs && borrow; l++) {
        const uint64_t old = N[l];
        N[l] = old - borrow;
        borrow = old < borrow ? 1 : 0;
      }
    }
    uint64_t yc = xc >> E::t, yp = xp >> E::t;
    for (int l = 0; l < kMaxLimbs; l++) {
      uint64_t wd = N[l];
      while (wd) {
        const int b = __builtin_ctzll(wd) + 64 * l;
        wd &= wd - 1;
        const uint64_t* M = L + (size_t)b * 4;
        const uint64_t nc = mulsum_mod<G>(M[0], yc, M[1], yp, pe, pc, p);
        const uint64_t np = mulsum_mod<G>(M[2], yc, M[3], yp, pe, pc, p);
        yc = nc; yp = np;
      }
    }
    xc = yc << E::t;
    xp = yp << E::t;
  } else {
    for (int l = 0; l < kMaxLimbs; l++) {
      uint64_t wd = N[l];
      while (wd) {
        const int b = __builtin_ctzll(wd) + 64 * l;
        wd &= wd - 1;
        const uint64_t* M = L + (size_t)b * 4;
        const uint64_t nc = mulsum_mod<G>(M[0], xc, M[1], xp, pe, pc, p);
        const uint64_t np = mulsum_mod<G>(M[2], xc, M[3], xp, pe, pc, p);
        xc = nc; xp = np;
      }
    }
  }
}

// Block splitting with the default variant: move (xc, xp) id 2^e steps on,
// e = kGmByteE[G], with one byte-table matrix per nonzero byte of id (tab:
// this generator's [8][256][4] slice).  Composite moduli first collapse (n0
// exact steps, unless already collapsed) and then also take M^(-n0) (neg),
// so the total stays id 2^e steps; id = 0 leaves the element as it is.
template <int G>
__device__ __forceinline__ void jump_bytes_elem(uint64_t& xc, uint64_t& xp, uint64_t id,
                                                const uint64_t* __restrict__ tab, const uint64_t* __restrict__ neg) {
  using E = Eng<G>;
  if (!id) return;
  int pe;
  uint64_t pc;
  prime_form(G, pe, pc);
  const uint64_t p = kGmParams[G].p;
  bool back = false;
  if constexpr (E::kComposite) {
    if (!(E::collapsed(xc) && E::collapsed(xp))) {
      for (int i = 0; i < kGmParams[G].n0; i++) { const uint64_t nx = E::slow_step(xc, xp); xp = xc; xc = nx; }
      back = true;
    }
  }
  constexpr int t = kGmParams[G].t;   // 2-adic exponent of the modulus (0: prime)
  uint64_t yc = xc >> t, yp = xp >> t;
  auto apply = [&](const uint64_t* M) {
    const uint64_t nc = mulsum_mod<G>(M[0], yc, M[1], yp, pe, pc, p);
    const uint64_t np = mulsum_mod<G>(M[2], yc, M[3], yp, pe, pc, p);
    yc = nc;
    yp = np;
  };
  for (int j = 0; j < 8; j++) {
    const uint32_t d = (uint32_t)(id >> (8 * j)) & 255u;
    if (d) apply(tab + ((size_t)j * 256 + d) * 4);
  }
  if (back) apply(neg);
  xc = yc << t;
  xp = yp << t;
}

// GQ58.3: a distance of N words from word offset `off` inside an 8-step
// block: (off + N) = 9 B + rem; N becomes 8 B ensemble steps, *new_off = rem.
__device__ __forceinline__ void gq3_words_to_steps(uint64_t* N, uint32_t off, uint32_t* new_off) {
  uint64_t carry = off;
  for (int l = 0; l <= kMaxLimbs && carry; l++) {
    const uint64_t old = N[l];
    N[l] = old + carry;
    carry = N[l] < old ? 1 : 0;
  }
  uint64_t r = 0;   // divide by 9 in 32-bit pieces
  for (int l = kMaxLimbs; l >= 0; l--) {
    const uint64_t hi = (r << 32) | (N[l] >> 32);
    const uint64_t qh = hi / 9;
    r = hi % 9;
    const uint64_t lo = (r << 32) | (N[l] & 0xFFFFFFFFull);
    const uint64_t ql = lo / 9;
    r = lo % 9;
    N[l] = (qh << 32) | ql;
  }
  *new_off = (uint32_t)r;
  uint64_t c3 = 0;   // times 8
  for (int l = 0; l <= kMaxLimbs; l++) {
    const uint64_t v = N[l];
    N[l] = (v << 3) | c3;
    c3 = v >> 61;
  }
}

// Load element e of *in and move it `start` outputs ahead (start < 2^64).
// Returns the word offset inside the GQ58.3 block (0 for the others).
// kJump = false: the caller guarantees start == 0 (no jump code is built).
template <int G, bool kJump = true>
__device__ __forceinline__ uint32_t load_at(const GmState* in, int e, uint64_t start, uint64_t& xc, uint64_t& xp,
                                            const uint64_t* __restrict__ ladder) {
  xc = in->xc[e];
  xp = in->xp[e];
  uint32_t off = (G == 6) ? in->off : 0;
  if (kJump && start) {
    uint64_t N[kMaxLimbs + 1];
    for (int l = 0; l <= kMaxLimbs; l++) N[l] = 0;
    N[0] = start;
    if (G == 6) gq3_words_to_steps(N, off, &off);
    jump_steps_elem<G>(xc, xp, N, ladder);
  }
  return off;
}

// ---------------------------------------------- v = 1, s = 32: ballots
// Each half-wavefront is one section: element e = 31 - (lane & 31) of state
// *in moved `start` outputs ahead, n outputs to out, advanced state to *sout
// (none when sout is null).
// n must be the same for both halves (the ballot spans the wavefront); a dead
// half (live = false) follows along without loads or stores.
template <int G, int DT, bool kJump = true>
__device__ __forceinline__ void gen32_wave(bool live, const GmState* in, uint64_t start, uint64_t n, void* out,
                                           GmState* sout, const uint64_t* __restrict__ ladder) {
  const int li = threadIdx.x & 31;        // bit position of this element's digit
  const int e = 31 - li;                  // element index
  uint64_t xc = 0, xp = 0;
  if (live) load_at<G, kJump>(in, e, start, xc, xp, ladder);
  Elem<G> el;
  el.load(xc, xp);
  // the word of step u goes to lane u of each half of the wavefront: a
  // full block of 32 steps writes the ballot halves with v_writelane, a
  // ragged last block selects per lane
  const bool upper = (threadIdx.x & 32) != 0;
  uint32_t keep = 0;
  for (uint64_t t0 = 0; t0 < n; t0 += 32) {
    const int m = (n - t0) < 32 ? (int)(n - t0) : 32;
    if (m == 32) {
      el.block([&](auto stepf) {
        static_for<0, 32>([&](auto uc) {
          constexpr int u = decltype(uc)::value;
          const uint64_t mask = __ballot(stepf());
          keep = writelane_pair<u>(keep, (uint32_t)mask, (uint32_t)(mask >> 32));
        });
      });
    } else {
      for (int u = 0; u < m; u++) {
        el.maybe_switch();
        const uint64_t mask = __ballot(el.step());
        const uint32_t w = upper ? (uint32_t)(mask >> 32) : (uint32_t)mask;
        keep = (u == li) ? w : keep;
      }
    }
    if (live && li < m) put<DT>(out, t0 + li, keep);
  }
  if (live && sout) {
    el.get(xc, xp);
    sout->xc[e] = xc;
    sout->xp[e] = xp;
    if (li == 0) { sout->off = 0; sout->pad = 0; }
  }
}

}  // namespace gm
}  // namespace prand
