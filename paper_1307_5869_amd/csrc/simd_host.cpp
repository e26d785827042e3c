// CPU SIMD generation (paper, section "Generation with SSE": a SIMD state is
// obtained from a plain state with rng_get_sse_state_, and rng_sse_generate_
// returns the next 32-bit output of the same sequence).  Host code only, for
// x86-64 with AVX2 and FMA (checked at run time; without them, or with
// PRAND_SIMD_DISABLE set when the state is made, the same buffers are filled
// by plain scalar code).  The outputs equal those of the plain state,
// word for word.
//
// Every generator refills a buffer of outputs at a time:
//   MT19937   the 624-word block twisted eight words per instruction (the
//             words the recurrence reads across the 227-word boundary come
//             from an eight-word mirror of the block's first renewed words)
//             and tempered eight at a time: one refill = one block.
//   LFSR113   eight lanes, lane j holding the state j L outputs after the
//             buffer start (L = kLaneLen), so one refill holds 8 L outputs in
//             sequence order; the four components of eight lanes step in
//             four 8 x 32-bit registers, and every eight steps an 8 x 8
//             transpose puts each lane's words in its part of the buffer.
//             After a refill lane j stands (j + 1) L on and is jumped 7 L
//             further (one F2 matrix per component).
//   MRG32K3A  four lanes in the same way, the two recurrences in FP64 on
//             centred residues (r = p - m rint(p / m): products below 2^53,
//             no correction step), the output map in 32-bit integers.
//   GM/GQ     the ensemble's elements in the lanes of 4 x 64-bit registers.
//             After the collapse (every element of a composite modulus
//             g = 2^t p divisible by 2^t; prime moduli from the start) an
//             element is y = x / 2^t and steps y' = k y_c - q y_p mod p,
//             p = 2^e - c, as a sum of 32 x 32-bit products folded with
//             2^e = c (mod p); the digits floor(2^v y / p) are read off y
//             (v = 1: one compare per element, and the compare masks of
//             eight registers are the word; v = 3, 4: the top v bits of y
//             and one correcting compare).  Steps before the collapse are
//             exact scalar steps mod g.
//
// The state blob is opaque to the caller (prand_simd_state_bytes bytes, any
// alignment: the code uses unaligned vector loads and stores).
#include <immintrin.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "prand.h"

namespace prand {
// section-start tables of the many-stream kernels, reused here for the lane
// jumps (row j - 1: the jump by j L), from tables.cpp
void build_mrg_section_table(uint64_t seclen, uint32_t* out);
void build_lfsr_section_table(uint64_t seclen, uint32_t* out);
}  // namespace prand

namespace {

typedef unsigned __int128 u128;

constexpr uint32_t kMagic = 0x53494d44u;   // "SIMD"
constexpr int kLaneLen = 512;               // outputs per lane per refill (LFSR113, MRG32K3A)
constexpr int kSecRows = 63;

struct Header {
  uint32_t magic;
  int32_t gen;
  uint32_t pos, len;   // next buffer word, words in the buffer
  uint32_t vec;        // 1: AVX2 path, 0: scalar path
  uint32_t pad[3];
};

struct MtPart {
  uint32_t mt[624 + 8];   // the current block, then a mirror of its first eight words
  uint32_t buf[624];
};
struct LfsrPart {
  uint32_t z[4][8];       // component c of lane j
  uint32_t buf[8 * kLaneLen];
};
struct MrgPart {
  double x[3][4], y[3][4];   // centred residues: x_n, x_{n-1}, x_{n-2} of lane j
  uint32_t buf[4 * kLaneLen];
};
constexpr int kGmBuf = 1152;   // 1024 v = 1/4 steps, or 128 GQ58.3 blocks of 9 words
struct GmPart {
  uint64_t c[32], p[32];   // x^(n) and x^(n-1): exact residues mod g before the collapse, y = x / 2^t after
  uint32_t collapsed;
  uint32_t pad;
  uint32_t buf[kGmBuf];
};

struct SimdState {
  Header h;
  union {
    MtPart mt;
    LfsrPart lf;
    MrgPart mrg;
    GmPart gm;
  };
};

// ------------------------------------------------------------- parameters
struct GmP {
  uint64_t k, q, p;   // recurrence constants, prime modulus p = 2^e - c
  int e;
  uint64_t c;
  int t, v, s;        // g = 2^t p; digit bits; ensemble size
};
GmP gm_params(int gen) {
  switch (gen) {
    case PRAND_GM19: return {15, 28, 524287ull, 19, 1, 0, 1, 32};
    case PRAND_GM29: return {4, 2, 536870909ull, 29, 3, 0, 1, 32};
    case PRAND_GM31: return {11, 14, 2147483647ull, 31, 1, 0, 1, 32};
    case PRAND_GM55: return {256, 176, 2251799813685119ull, 51, 129, 4, 4, 8};
    case PRAND_GM61: return {24, 74, 2305843009213693951ull, 61, 1, 0, 1, 32};
    case PRAND_GQ58X1: return {8, 48, 536870909ull, 29, 3, 29, 1, 32};
    case PRAND_GQ58X3: return {8, 48, 536870909ull, 29, 3, 29, 3, 12};
    default: return {8, 48, 536870909ull, 29, 3, 29, 4, 8};
  }
}

bool cpu_has_avx2() {
  static const bool ok = __builtin_cpu_supports("avx2") && __builtin_cpu_supports("fma");
  return ok;
}

// ------------------------------------------------------------------ MT19937
inline uint32_t temper(uint32_t y) {
  y ^= y >> 11;
  y ^= (y << 7) & 0x9D2C5680u;
  y ^= (y << 15) & 0xEFC60000u;
  return y ^ (y >> 18);
}

void mt_refill_scalar(MtPart& m) {
  for (int j = 0; j < 624; j++) {
    const uint32_t y = (m.mt[j] & 0x80000000u) | (m.mt[j == 623 ? 0 : j + 1] & 0x7FFFFFFFu);
    const int o = j + 397 < 624 ? j + 397 : j + 397 - 624;
    m.mt[j] = m.mt[o] ^ (y >> 1) ^ ((y & 1u) ? 0x9908B0DFu : 0u);
  }
  for (int j = 0; j < 624; j++) m.buf[j] = temper(m.mt[j]);
}

__attribute__((target("avx2"))) inline __m256i mt_vec(__m256i a, __m256i b, __m256i c) {
  const __m256i up = _mm256_set1_epi32((int)0x80000000u), lo = _mm256_set1_epi32(0x7FFFFFFF);
  const __m256i y = _mm256_or_si256(_mm256_and_si256(a, up), _mm256_and_si256(b, lo));
  const __m256i odd = _mm256_and_si256(y, _mm256_set1_epi32(1));
  const __m256i mag = _mm256_and_si256(_mm256_sub_epi32(_mm256_setzero_si256(), odd),
                                       _mm256_set1_epi32((int)0x9908B0DFu));
  return _mm256_xor_si256(_mm256_xor_si256(c, _mm256_srli_epi32(y, 1)), mag);
}

__attribute__((target("avx2"))) inline __m256i ld(const uint32_t* p) {
  return _mm256_loadu_si256((const __m256i*)p);
}

__attribute__((target("avx2"))) void mt_refill_avx2(MtPart& m) {
  uint32_t* mt = m.mt;
  // words 0..223: every word read is an old one
  for (int i = 0; i < 224; i += 8) {
    const __m256i v = mt_vec(ld(mt + i), ld(mt + i + 1), ld(mt + i + 397));
    _mm256_storeu_si256((__m256i*)(mt + i), v);
    if (i == 0) _mm256_storeu_si256((__m256i*)(mt + 624), v);   // mirror of the renewed words 0..7
  }
  // words 224..231: words 224..226 read old words 621..623, words 227..231
  // the renewed words 0..4, which the mirror holds at 624..628
  _mm256_storeu_si256((__m256i*)(mt + 224), mt_vec(ld(mt + 224), ld(mt + 225), ld(mt + 621)));
  // words 232..623 read renewed words j - 227; word 623 pairs with the
  // renewed word 0 (mirror slot 624)
  for (int i = 232; i < 624; i += 8)
    _mm256_storeu_si256((__m256i*)(mt + i), mt_vec(ld(mt + i), ld(mt + i + 1), ld(mt + i - 227)));
  const __m256i b1 = _mm256_set1_epi32((int)0x9D2C5680u), b2 = _mm256_set1_epi32((int)0xEFC60000u);
  for (int i = 0; i < 624; i += 8) {
    __m256i y = ld(mt + i);
    y = _mm256_xor_si256(y, _mm256_srli_epi32(y, 11));
    y = _mm256_xor_si256(y, _mm256_and_si256(_mm256_slli_epi32(y, 7), b1));
    y = _mm256_xor_si256(y, _mm256_and_si256(_mm256_slli_epi32(y, 15), b2));
    y = _mm256_xor_si256(y, _mm256_srli_epi32(y, 18));
    _mm256_storeu_si256((__m256i*)(m.buf + i), y);
  }
}

// ------------------------------------------------------------------ LFSR113
constexpr uint32_t kLfMask[4] = {0xFFFFFFFEu, 0xFFFFFFF8u, 0xFFFFFFF0u, 0xFFFFFF80u};
constexpr int kLfQ[4] = {6, 2, 13, 3};
constexpr int kLfSh[4] = {13, 27, 21, 12};
constexpr int kLfS[4] = {18, 2, 7, 13};

inline uint32_t lfsr_comp(uint32_t z, int c) {
  return ((z & kLfMask[c]) << kLfS[c]) ^ (((z << kLfQ[c]) ^ z) >> kLfSh[c]);
}

uint32_t f2_apply(const uint32_t* cols, uint32_t v) {
  uint32_t r = 0;
  for (int j = 0; j < 32; j++) r ^= cols[j] & (0u - ((v >> j) & 1u));
  return r;
}

// section-start tables for L = kLaneLen, built once per process
const uint32_t* lfsr_lane_table() {
  static uint32_t tab[kSecRows * 128];
  static std::once_flag once;
  std::call_once(once, [] { prand::build_lfsr_section_table(kLaneLen, tab); });
  return tab;
}
const uint32_t* mrg_lane_table() {
  static uint32_t tab[kSecRows * 18];
  static std::once_flag once;
  std::call_once(once, [] { prand::build_mrg_section_table(kLaneLen, tab); });
  return tab;
}

void lfsr_jump_lane(LfsrPart& l, int j, const uint32_t* row) {
  for (int c = 0; c < 4; c++) l.z[c][j] = f2_apply(row + 32 * c, l.z[c][j]);
}

void lfsr_refill_scalar(LfsrPart& l) {
  for (int j = 0; j < 8; j++) {
    uint32_t z[4] = {l.z[0][j], l.z[1][j], l.z[2][j], l.z[3][j]};
    for (int t = 0; t < kLaneLen; t++) {
      for (int c = 0; c < 4; c++) z[c] = lfsr_comp(z[c], c);
      l.buf[j * kLaneLen + t] = z[0] ^ z[1] ^ z[2] ^ z[3];
    }
    for (int c = 0; c < 4; c++) l.z[c][j] = z[c];
  }
}

// 8 x 8 transpose of 32-bit words: r[i] lane j <- r[j] lane i
__attribute__((target("avx2"))) inline void transpose8(__m256i r[8]) {
  __m256i t[8], u[8];
  for (int i = 0; i < 8; i += 2) {
    t[i] = _mm256_unpacklo_epi32(r[i], r[i + 1]);
    t[i + 1] = _mm256_unpackhi_epi32(r[i], r[i + 1]);
  }
  for (int i = 0; i < 8; i += 4) {
    u[i] = _mm256_unpacklo_epi64(t[i], t[i + 2]);
    u[i + 1] = _mm256_unpackhi_epi64(t[i], t[i + 2]);
    u[i + 2] = _mm256_unpacklo_epi64(t[i + 1], t[i + 3]);
    u[i + 3] = _mm256_unpackhi_epi64(t[i + 1], t[i + 3]);
  }
  for (int i = 0; i < 4; i++) {
    r[i] = _mm256_permute2x128_si256(u[i], u[i + 4], 0x20);
    r[i + 4] = _mm256_permute2x128_si256(u[i], u[i + 4], 0x31);
  }
}

template <int C>
__attribute__((target("avx2"))) inline __m256i lfsr_vcomp(__m256i z) {
  const __m256i a = _mm256_slli_epi32(_mm256_and_si256(z, _mm256_set1_epi32((int)kLfMask[C])), kLfS[C]);
  const __m256i b = _mm256_srli_epi32(_mm256_xor_si256(_mm256_slli_epi32(z, kLfQ[C]), z), kLfSh[C]);
  return _mm256_xor_si256(a, b);
}

__attribute__((target("avx2"))) void lfsr_refill_avx2(LfsrPart& l) {
  __m256i z0 = _mm256_loadu_si256((const __m256i*)l.z[0]), z1 = _mm256_loadu_si256((const __m256i*)l.z[1]);
  __m256i z2 = _mm256_loadu_si256((const __m256i*)l.z[2]), z3 = _mm256_loadu_si256((const __m256i*)l.z[3]);
  for (int t = 0; t < kLaneLen; t += 8) {
    __m256i r[8];
    for (int k = 0; k < 8; k++) {
      z0 = lfsr_vcomp<0>(z0);
      z1 = lfsr_vcomp<1>(z1);
      z2 = lfsr_vcomp<2>(z2);
      z3 = lfsr_vcomp<3>(z3);
      r[k] = _mm256_xor_si256(_mm256_xor_si256(z0, z1), _mm256_xor_si256(z2, z3));   // step k, lane j
    }
    transpose8(r);   // r[j]: lane j, steps t .. t + 7
    for (int j = 0; j < 8; j++) _mm256_storeu_si256((__m256i*)(l.buf + j * kLaneLen + t), r[j]);
  }
  _mm256_storeu_si256((__m256i*)l.z[0], z0);
  _mm256_storeu_si256((__m256i*)l.z[1], z1);
  _mm256_storeu_si256((__m256i*)l.z[2], z2);
  _mm256_storeu_si256((__m256i*)l.z[3], z3);
}

// after a refill lane j stands (j + 1) L after the buffer start; the next
// buffer starts 8 L after it, so every lane moves 7 L on
void lfsr_advance_lanes(LfsrPart& l) {
  const uint32_t* row = lfsr_lane_table() + 6 * 128;
  for (int j = 0; j < 8; j++) lfsr_jump_lane(l, j, row);
}

// ----------------------------------------------------------------- MRG32K3A
constexpr uint64_t kM1 = 4294967087ull, kM2 = 4294944443ull;

void mat3_apply(const uint32_t* M, uint64_t m, uint64_t v[3]) {
  uint64_t r[3];
  for (int i = 0; i < 3; i++) {
    u128 acc = 0;
    for (int k = 0; k < 3; k++) acc += (u128)M[3 * i + k] * v[k];
    r[i] = (uint64_t)(acc % m);
  }
  v[0] = r[0];
  v[1] = r[1];
  v[2] = r[2];
}

inline double centre(uint64_t v, double m) { return (double)v > 0.5 * m ? (double)v - m : (double)v; }
inline uint64_t canon(double r, uint64_t m) { return r < 0 ? (uint64_t)(int64_t)r + m : (uint64_t)r; }

void mrg_lane_get(const MrgPart& g, int j, uint64_t x[3], uint64_t y[3]) {
  for (int i = 0; i < 3; i++) {
    x[i] = canon(g.x[i][j], kM1);
    y[i] = canon(g.y[i][j], kM2);
  }
}
void mrg_lane_set(MrgPart& g, int j, const uint64_t x[3], const uint64_t y[3]) {
  for (int i = 0; i < 3; i++) {
    g.x[i][j] = centre(x[i], (double)kM1);
    g.y[i][j] = centre(y[i], (double)kM2);
  }
}
void mrg_jump_lane(MrgPart& g, int j, const uint32_t* row) {
  uint64_t x[3], y[3];
  mrg_lane_get(g, j, x, y);
  mat3_apply(row, kM1, x);
  mat3_apply(row + 9, kM2, y);
  mrg_lane_set(g, j, x, y);
}

void mrg_refill_scalar(MrgPart& g) {
  for (int j = 0; j < 4; j++) {
    uint64_t x[3], y[3];
    mrg_lane_get(g, j, x, y);
    for (int t = 0; t < kLaneLen; t++) {
      const uint64_t nx = (1403580ull * x[1] + 810728ull * (kM1 - x[2])) % kM1;
      const uint64_t ny = (527612ull * y[0] + 1370589ull * (kM2 - y[2])) % kM2;
      x[2] = x[1]; x[1] = x[0]; x[0] = nx;
      y[2] = y[1]; y[1] = y[0]; y[0] = ny;
      g.buf[j * kLaneLen + t] = (uint32_t)(nx > ny ? nx - ny : nx + kM1 - ny);
    }
    mrg_lane_set(g, j, x, y);
  }
}

__attribute__((target("avx2,fma"))) inline __m256d mrg_reduce(__m256d p, __m256d m, __m256d inv) {
  const __m256d k = _mm256_round_pd(_mm256_mul_pd(p, inv), _MM_FROUND_TO_NEAREST_INT | _MM_FROUND_NO_EXC);
  return _mm256_fnmadd_pd(k, m, p);
}
// canonical residue (32-bit) of a centred one, m = 2^32 - C
template <uint32_t C>
__attribute__((target("avx2"))) inline __m128i mrg_canon(__m256d r) {
  const __m128i i = _mm256_cvtpd_epi32(r);   // exact: |r| < 2^31
  return _mm_sub_epi32(i, _mm_and_si128(_mm_srai_epi32(i, 31), _mm_set1_epi32((int)C)));
}

__attribute__((target("avx2,fma"))) void mrg_refill_avx2(MrgPart& g) {
  __m256d x0 = _mm256_loadu_pd(g.x[0]), x1 = _mm256_loadu_pd(g.x[1]), x2 = _mm256_loadu_pd(g.x[2]);
  __m256d y0 = _mm256_loadu_pd(g.y[0]), y1 = _mm256_loadu_pd(g.y[1]), y2 = _mm256_loadu_pd(g.y[2]);
  const __m256d a12 = _mm256_set1_pd(1403580.0), a13 = _mm256_set1_pd(-810728.0);
  const __m256d a21 = _mm256_set1_pd(527612.0), a23 = _mm256_set1_pd(-1370589.0);
  const __m256d m1 = _mm256_set1_pd((double)kM1), m2 = _mm256_set1_pd((double)kM2);
  const __m256d i1 = _mm256_set1_pd(1.0 / (double)kM1), i2 = _mm256_set1_pd(1.0 / (double)kM2);
  const __m128i sign = _mm_set1_epi32((int)0x80000000u), c209 = _mm_set1_epi32(209);
  for (int t = 0; t < kLaneLen; t += 4) {
    __m128i r[4];
    for (int k = 0; k < 4; k++) {
      const __m256d x = mrg_reduce(_mm256_fmadd_pd(a12, x1, _mm256_mul_pd(a13, x2)), m1, i1);
      const __m256d y = mrg_reduce(_mm256_fmadd_pd(a21, y0, _mm256_mul_pd(a23, y2)), m2, i2);
      x2 = x1; x1 = x0; x0 = x;
      y2 = y1; y1 = y0; y0 = y;
      const __m128i xc = mrg_canon<209u>(x), yc = mrg_canon<22853u>(y);
      const __m128i d = _mm_sub_epi32(xc, yc);
      // x > y (unsigned): d, else d - 209 (= x - y + m1 mod 2^32)
      const __m128i gt = _mm_cmpgt_epi32(_mm_xor_si128(xc, sign), _mm_xor_si128(yc, sign));
      r[k] = _mm_sub_epi32(d, _mm_andnot_si128(gt, c209));   // step k, lane j
    }
    // 4 x 4 transpose: r[j] = lane j, steps t .. t + 3
    const __m128i t0 = _mm_unpacklo_epi32(r[0], r[1]), t1 = _mm_unpackhi_epi32(r[0], r[1]);
    const __m128i t2 = _mm_unpacklo_epi32(r[2], r[3]), t3 = _mm_unpackhi_epi32(r[2], r[3]);
    r[0] = _mm_unpacklo_epi64(t0, t2);
    r[1] = _mm_unpackhi_epi64(t0, t2);
    r[2] = _mm_unpacklo_epi64(t1, t3);
    r[3] = _mm_unpackhi_epi64(t1, t3);
    for (int j = 0; j < 4; j++) _mm_storeu_si128((__m128i*)(g.buf + j * kLaneLen + t), r[j]);
  }
  _mm256_storeu_pd(g.x[0], x0); _mm256_storeu_pd(g.x[1], x1); _mm256_storeu_pd(g.x[2], x2);
  _mm256_storeu_pd(g.y[0], y0); _mm256_storeu_pd(g.y[1], y1); _mm256_storeu_pd(g.y[2], y2);
}

void mrg_advance_lanes(MrgPart& g) {
  const uint32_t* row = mrg_lane_table() + 2 * 18;   // the jump by 3 L
  for (int j = 0; j < 4; j++) mrg_jump_lane(g, j, row);
}

// GQ58.3: the 36-bit steps of a block, most significant first, cut into
// nine 32-bit words (at most 67 bits are pending at a time)
struct BitSink {
  u128 acc = 0;
  int nb = 0;
  uint32_t* out;
  explicit BitSink(uint32_t* o) : out(o) {}
  void put(uint64_t chunk36) {
    acc = (acc << 36) | chunk36;
    nb += 36;
    while (nb >= 32) {
      *out++ = (uint32_t)(acc >> (nb - 32));
      nb -= 32;
      acc &= (((u128)1) << nb) - 1;
    }
  }
};

// -------------------------------------------------------------------- GM/GQ
// exact scalar step mod g = 2^t p (every product sum below 2^64 except for
// GM61, prime, which folds a 128-bit sum)
uint64_t gm_exact_step(const GmP& P, uint64_t xc, uint64_t xp) {
  const uint64_t g = P.p << P.t;
  if (P.e == 61) {
    const u128 t = (u128)P.k * xc + (u128)P.q * (g - xp);
    const uint64_t lo = (uint64_t)t, hi = (uint64_t)(t >> 64);
    uint64_t r = (lo & g) + ((lo >> 61) | (hi << 3));
    r = (r & g) + (r >> 61);
    return r >= g ? r - g : r;
  }
  return (P.k * xc + P.q * (g - xp)) % g;
}

// y' = k yc - q yp mod p on collapsed elements (y < p)
inline uint64_t gm_step_y(const GmP& P, uint64_t yc, uint64_t yp) {
  const u128 t = (u128)P.k * yc + (u128)P.q * (2 * P.p - yp);
  return (uint64_t)(t % P.p);
}
inline uint64_t gm_digit(const GmP& P, uint64_t y) { return (uint64_t)(((u128)y << P.v) / P.p); }

bool gm_all_collapsed(const GmP& P, const GmPart& G) {
  if (P.t == 0) return true;
  const uint64_t m = (1ull << P.t) - 1;
  for (int i = 0; i < P.s; i++)
    if ((G.c[i] & m) || (G.p[i] & m)) return false;
  return true;
}
void gm_to_collapsed(const GmP& P, GmPart& G) {
  for (int i = 0; i < P.s; i++) {
    G.c[i] >>= P.t;
    G.p[i] >>= P.t;
  }
  G.collapsed = 1;
}

// one step of the whole ensemble, scalar: the s v digit bits (element 0
// most significant)
uint64_t gm_step_scalar(const GmP& P, GmPart& G) {
  uint64_t bits = 0;
  for (int i = 0; i < P.s; i++) {
    uint64_t nx, d;
    if (G.collapsed) {
      nx = gm_step_y(P, G.c[i], G.p[i]);
      d = gm_digit(P, nx);
    } else {
      nx = gm_exact_step(P, G.c[i], G.p[i]);
      d = (uint64_t)(((u128)nx << P.v) / ((u128)P.p << P.t));
    }
    G.p[i] = G.c[i];
    G.c[i] = nx;
    bits = (bits << P.v) | d;
  }
  if (!G.collapsed && gm_all_collapsed(P, G)) gm_to_collapsed(P, G);
  return bits;
}

// Vector step of four collapsed elements: y' = (k yc + q (2p - yp)) mod p.
// For e <= 31 both products fit 32 x 32 -> 64 bits; for e = 51 and 61 the
// operands are split at bit 32 and the high part's 2^32 factor is folded
// with 2^e = c (mod p).
template <int E>
__attribute__((target("avx2"))) inline __m256i gm_vstep(__m256i yc, __m256i yp, __m256i kv, __m256i qv, __m256i p2,
                                                      __m256i pv, __m256i cv) {
  const __m256i s = _mm256_sub_epi64(p2, yp);   // 2p - yp, in (p, 2p]
  const __m256i mask = _mm256_set1_epi64x((long long)((1ull << E) - 1));
  __m256i t;
  if constexpr (E <= 31) {
    t = _mm256_add_epi64(_mm256_mul_epu32(kv, yc), _mm256_mul_epu32(qv, s));   // < 2^40
  } else {
    const __m256i hi = _mm256_add_epi64(_mm256_mul_epu32(kv, _mm256_srli_epi64(yc, 32)),
                                        _mm256_mul_epu32(qv, _mm256_srli_epi64(s, 32)));
    const __m256i lo = _mm256_add_epi64(_mm256_mul_epu32(kv, yc), _mm256_mul_epu32(qv, s));   // low halves
    // hi 2^32 = (hi >> (E - 32)) 2^E + (hi mod 2^(E-32)) 2^32 = (hi >> (E - 32)) c + ...
    const __m256i hm = _mm256_set1_epi64x((long long)((1ull << (E - 32)) - 1));
    t = _mm256_add_epi64(_mm256_add_epi64(_mm256_slli_epi64(_mm256_and_si256(hi, hm), 32), lo),
                         _mm256_mul_epu32(_mm256_srli_epi64(hi, E - 32), cv));
  }
  // two folds with 2^E = c, then one conditional subtraction
  t = _mm256_add_epi64(_mm256_and_si256(t, mask), _mm256_mul_epu32(_mm256_srli_epi64(t, E), cv));
  t = _mm256_add_epi64(_mm256_and_si256(t, mask), _mm256_mul_epu32(_mm256_srli_epi64(t, E), cv));
  const __m256i ge = _mm256_cmpgt_epi64(t, _mm256_sub_epi64(pv, _mm256_set1_epi64x(1)));
  return _mm256_sub_epi64(t, _mm256_and_si256(ge, pv));
}

// floor(2^V y / p), p = 2^E - c: the top V bits d0 of y, plus one when
// 2^V y >= (d0 + 1) p
template <int E, int V>
__attribute__((target("avx2"))) inline __m256i gm_vdigit(__m256i y, __m256i cv) {
  const __m256i d0 = _mm256_srli_epi64(y, E - V);
  const __m256i d1 = _mm256_add_epi64(d0, _mm256_set1_epi64x(1));
  const __m256i diff = _mm256_add_epi64(_mm256_sub_epi64(_mm256_slli_epi64(y, V), _mm256_slli_epi64(d1, E)),
                                        _mm256_mul_epu32(d1, cv));
  const __m256i neg = _mm256_cmpgt_epi64(_mm256_setzero_si256(), diff);   // diff < 0: d0
  return _mm256_add_epi64(d0, _mm256_andnot_si256(neg, _mm256_set1_epi64x(1)));
}

// v = 1, s = 32: the elements sit in reverse order (vector r lane l =
// element 31 - 4 r - l), so compare mask bit 4 r + l is the digit of element
// 31 - (4 r + l), i.e. word bit 4 r + l.  Fills `count` words.
template <int E>
__attribute__((target("avx2"))) void gm_v1_avx2(const GmP& P, GmPart& G, uint32_t* out, int count) {
  __m256i c[8], p[8];
  for (int r = 0; r < 8; r++) {
    alignas(32) uint64_t tc[4], tp[4];
    for (int l = 0; l < 4; l++) {
      tc[l] = G.c[31 - 4 * r - l];
      tp[l] = G.p[31 - 4 * r - l];
    }
    c[r] = _mm256_load_si256((const __m256i*)tc);
    p[r] = _mm256_load_si256((const __m256i*)tp);
  }
  const __m256i kv = _mm256_set1_epi64x((long long)P.k), qv = _mm256_set1_epi64x((long long)P.q);
  const __m256i pv = _mm256_set1_epi64x((long long)P.p), p2 = _mm256_set1_epi64x((long long)(2 * P.p));
  const __m256i cv = _mm256_set1_epi64x((long long)P.c);
  const __m256i half = _mm256_set1_epi64x((long long)((P.p - 1) / 2));   // y > (p - 1) / 2: digit 1
  for (int w = 0; w < count; w++) {
    uint32_t word = 0;
    for (int r = 0; r < 8; r++) {
      const __m256i n = gm_vstep<E>(c[r], p[r], kv, qv, p2, pv, cv);
      p[r] = c[r];
      c[r] = n;
      word |= (uint32_t)_mm256_movemask_pd(_mm256_castsi256_pd(_mm256_cmpgt_epi64(n, half))) << (4 * r);
    }
    out[w] = word;
  }
  for (int r = 0; r < 8; r++) {
    alignas(32) uint64_t tc[4], tp[4];
    _mm256_store_si256((__m256i*)tc, c[r]);
    _mm256_store_si256((__m256i*)tp, p[r]);
    for (int l = 0; l < 4; l++) {
      G.c[31 - 4 * r - l] = tc[l];
      G.p[31 - 4 * r - l] = tp[l];
    }
  }
}

// v = 3 or 4: elements in order (vector r lane l = element 4 r + l); the
// digits are shifted to their place in the step's s v bits and OR-ed.
// V = 4 (s = 8): one word per step.  V = 3 (s = 12): 36 bits per step; a
// block of 8 steps gives 9 words.  Fills `count` steps (V = 4) or blocks.
template <int E, int V>
__attribute__((target("avx2"))) void gm_vwide_avx2(const GmP& P, GmPart& G, uint32_t* out, int count) {
  constexpr int NV = (V == 3) ? 3 : 2;
  constexpr int S = 4 * NV;
  __m256i c[NV], p[NV], sh[NV];
  for (int r = 0; r < NV; r++) {
    c[r] = _mm256_loadu_si256((const __m256i*)(G.c + 4 * r));
    p[r] = _mm256_loadu_si256((const __m256i*)(G.p + 4 * r));
    sh[r] = _mm256_set_epi64x(V * (S - 4 - 4 * r), V * (S - 3 - 4 * r), V * (S - 2 - 4 * r), V * (S - 1 - 4 * r));
  }
  const __m256i kv = _mm256_set1_epi64x((long long)P.k), qv = _mm256_set1_epi64x((long long)P.q);
  const __m256i pv = _mm256_set1_epi64x((long long)P.p), p2 = _mm256_set1_epi64x((long long)(2 * P.p));
  const __m256i cv = _mm256_set1_epi64x((long long)P.c);
  for (int u = 0; u < count; u++) {
    // a step (V = 4: one word) or a block of 8 steps (V = 3: nine words)
    BitSink sink(out + 9 * u);
    for (int k = 0; k < (V == 3 ? 8 : 1); k++) {
      __m256i acc = _mm256_setzero_si256();
      for (int r = 0; r < NV; r++) {
        const __m256i n = gm_vstep<E>(c[r], p[r], kv, qv, p2, pv, cv);
        p[r] = c[r];
        c[r] = n;
        acc = _mm256_or_si256(acc, _mm256_sllv_epi64(gm_vdigit<E, V>(n, cv), sh[r]));
      }
      const __m128i h = _mm_or_si128(_mm256_castsi256_si128(acc), _mm256_extracti128_si256(acc, 1));
      const uint64_t bits = (uint64_t)_mm_cvtsi128_si64(_mm_or_si128(h, _mm_unpackhi_epi64(h, h)));
      if (V == 3) sink.put(bits);
      else out[u] = (uint32_t)bits;
    }
  }
  for (int r = 0; r < NV; r++) {
    _mm256_storeu_si256((__m256i*)(G.c + 4 * r), c[r]);
    _mm256_storeu_si256((__m256i*)(G.p + 4 * r), p[r]);
  }
}

void gm_avx2(int gen, const GmP& P, GmPart& G, uint32_t* out, int count) {
  switch (gen) {
    case PRAND_GM19: gm_v1_avx2<19>(P, G, out, count); break;
    case PRAND_GM29: gm_v1_avx2<29>(P, G, out, count); break;
    case PRAND_GM31: gm_v1_avx2<31>(P, G, out, count); break;
    case PRAND_GM61: gm_v1_avx2<61>(P, G, out, count); break;
    case PRAND_GQ58X1: gm_v1_avx2<29>(P, G, out, count); break;
    case PRAND_GM55: gm_vwide_avx2<51, 4>(P, G, out, count); break;
    case PRAND_GQ58X3: gm_vwide_avx2<29, 3>(P, G, out, count); break;
    default: gm_vwide_avx2<29, 4>(P, G, out, count); break;
  }
}

// words of one unit of output (a step, or a GQ58.3 block of 8 steps),
// scalar; returns the words written
int gm_unit_scalar(const GmP& P, GmPart& G, uint32_t* out) {
  if (P.v != 3) {
    out[0] = (uint32_t)gm_step_scalar(P, G);
    return 1;
  }
  BitSink sink(out);
  for (int k = 0; k < 8; k++) sink.put(gm_step_scalar(P, G));
  return 9;
}

void gm_refill(SimdState& S) {
  const GmP P = gm_params(S.h.gen);
  GmPart& G = S.gm;
  const int units = P.v == 3 ? kGmBuf / 9 : kGmBuf;
  int u = 0, w = 0;
  // exact scalar steps until the ensemble has collapsed
  for (; u < units && !G.collapsed; u++) w += gm_unit_scalar(P, G, G.buf + w);
  if (u < units) {
    if (S.h.vec) {
      gm_avx2(S.h.gen, P, G, G.buf + w, units - u);
      w += (units - u) * (P.v == 3 ? 9 : 1);
    } else {
      for (; u < units; u++) w += gm_unit_scalar(P, G, G.buf + w);
    }
  }
  S.h.len = (uint32_t)w;
  S.h.pos = 0;
}

// ----------------------------------------------------------------- dispatch
void refill(SimdState& S) {
  switch (S.h.gen) {
    case PRAND_MT19937:
      if (S.h.vec) mt_refill_avx2(S.mt);
      else mt_refill_scalar(S.mt);
      S.h.len = 624;
      break;
    case PRAND_LFSR113:
      if (S.h.vec) lfsr_refill_avx2(S.lf);
      else lfsr_refill_scalar(S.lf);
      lfsr_advance_lanes(S.lf);
      S.h.len = 8 * kLaneLen;
      break;
    case PRAND_MRG32K3A:
      if (S.h.vec) mrg_refill_avx2(S.mrg);
      else mrg_refill_scalar(S.mrg);
      mrg_advance_lanes(S.mrg);
      S.h.len = 4 * kLaneLen;
      break;
    default:
      gm_refill(S);
      return;
  }
  S.h.pos = 0;
}

const uint32_t* buffer(const SimdState& S) {
  switch (S.h.gen) {
    case PRAND_MT19937: return S.mt.buf;
    case PRAND_LFSR113: return S.lf.buf;
    case PRAND_MRG32K3A: return S.mrg.buf;
    default: return S.gm.buf;
  }
}

SimdState* valid(void* p) {
  SimdState* S = (SimdState*)p;
  if (!S || S->h.magic != kMagic || S->h.gen < 0 || S->h.gen >= PRAND_NUM_GENERATORS) return nullptr;
  return S;
}

}  // namespace

extern "C" {

size_t prand_simd_state_bytes(void) { return sizeof(SimdState); }

int prand_get_simd_state(int gen, const void* h_state, void* simd_state) {
  if (gen < 0 || gen >= PRAND_NUM_GENERATORS || !h_state || !simd_state) return PRAND_EINVAL;
  SimdState& S = *(SimdState*)simd_state;
  std::memset(&S.h, 0, sizeof S.h);
  S.h.magic = kMagic;
  S.h.gen = gen;
  const char* off = std::getenv("PRAND_SIMD_DISABLE");
  S.h.vec = (cpu_has_avx2() && !(off && *off && *off != '0')) ? 1u : 0u;
  switch (gen) {
    case PRAND_MT19937: {
      uint32_t mt[624], idx;
      std::memcpy(mt, h_state, sizeof mt);
      std::memcpy(&idx, (const char*)h_state + sizeof mt, 4);
      if (idx > 624) idx = 624;
      std::memcpy(S.mt.mt, mt, sizeof mt);
      // the block's remaining words are the current buffer
      for (int j = 0; j < 624; j++) S.mt.buf[j] = temper(mt[j]);
      S.h.len = 624;
      S.h.pos = idx;
      return PRAND_OK;
    }
    case PRAND_LFSR113: {
      uint32_t z[4];
      std::memcpy(z, h_state, sizeof z);
      const uint32_t* tab = lfsr_lane_table();
      for (int c = 0; c < 4; c++) S.lf.z[c][0] = z[c];
      for (int j = 1; j < 8; j++) {
        for (int c = 0; c < 4; c++) S.lf.z[c][j] = z[c];
        lfsr_jump_lane(S.lf, j, tab + (size_t)(j - 1) * 128);
      }
      S.h.pos = S.h.len = 0;
      return PRAND_OK;
    }
    case PRAND_MRG32K3A: {
      uint32_t w[6];
      std::memcpy(w, h_state, sizeof w);
      const uint64_t x[3] = {w[0], w[1], w[2]}, y[3] = {w[3], w[4], w[5]};
      const uint32_t* tab = mrg_lane_table();
      for (int j = 0; j < 4; j++) {
        mrg_lane_set(S.mrg, j, x, y);
        if (j) mrg_jump_lane(S.mrg, j, tab + (size_t)(j - 1) * 18);
      }
      S.h.pos = S.h.len = 0;
      return PRAND_OK;
    }
    default: {
      const GmP P = gm_params(gen);
      const uint64_t* xp = (const uint64_t*)h_state;
      const uint64_t* xc = xp + 32;
      uint32_t offw;
      std::memcpy(&offw, (const char*)h_state + 512, 4);
      for (int i = 0; i < 32; i++) {
        S.gm.p[i] = i < P.s ? xp[i] : 0;
        S.gm.c[i] = i < P.s ? xc[i] : 0;
      }
      S.gm.collapsed = 0;
      if (gm_all_collapsed(P, S.gm)) gm_to_collapsed(P, S.gm);
      S.h.pos = S.h.len = 0;
      if (P.v == 3 && offw) {
        // the state stands at the start of a block whose first offw words
        // are used: make the block and skip them
        uint32_t blk[9];
        const int n = gm_unit_scalar(P, S.gm, blk);
        std::memcpy(S.gm.buf, blk, sizeof blk);
        S.h.len = (uint32_t)n;
        S.h.pos = offw < 9 ? offw : 9;
      }
      return PRAND_OK;
    }
  }
}

uint32_t prand_simd_next(void* simd_state) {
  SimdState* S = valid(simd_state);
  if (!S) return 0;
  if (S->h.pos >= S->h.len) refill(*S);
  return buffer(*S)[S->h.pos++];
}

int prand_simd_fill(void* simd_state, int dtype, void* h_out, uint64_t n) {
  SimdState* S = valid(simd_state);
  if (!S || (dtype != PRAND_U32 && dtype != PRAND_F32 && dtype != PRAND_F64) || (n && !h_out)) return PRAND_EINVAL;
  const bool mrg = S->h.gen == PRAND_MRG32K3A;
  uint64_t i = 0;
  while (i < n) {
    if (S->h.pos >= S->h.len) refill(*S);
    const uint32_t* b = buffer(*S) + S->h.pos;
    const uint64_t take = std::min<uint64_t>(S->h.len - S->h.pos, n - i);
    if (dtype == PRAND_U32) {
      std::memcpy((uint32_t*)h_out + i, b, take * 4);
    } else if (dtype == PRAND_F32) {
      float* o = (float*)h_out + i;
      for (uint64_t t = 0; t < take; t++) o[t] = (float)(b[t] >> 8) * 0x1p-24f;
    } else {
      double* o = (double*)h_out + i;
      const double norm = mrg ? 1.0 / 4294967088.0 : 0x1p-32;
      for (uint64_t t = 0; t < take; t++) o[t] = (double)b[t] * norm;
    }
    S->h.pos += (uint32_t)take;
    i += take;
  }
  return PRAND_OK;
}

int prand_simd_vectorized(const void* simd_state) {
  const SimdState* S = valid((void*)simd_state);
  return S ? (int)S->h.vec : PRAND_EINVAL;
}

}  // extern "C"
