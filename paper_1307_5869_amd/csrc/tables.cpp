// Context set-up: the jump-ahead ladders of MRG32K3A, LFSR113 and the GM/GQ
// ensembles, computed once on the host when a context is created and then
// uploaded (the MT19937 polynomials are built in mt_poly.cpp).  A distance is
// applied as one ladder entry M^(2^b) per set bit b (binary decomposition of
// the distance, as in the paper's jump-ahead sections).
#include <cstring>
#include <vector>

#include "prand_impl.h"

namespace prand {
namespace {

typedef unsigned __int128 u128;

// ---------------------------------------------------------------- MRG32K3A
void mat3_sqr(const uint64_t* a, uint64_t* r, uint64_t m) {
  uint64_t t[9];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      u128 acc = 0;
      for (int k = 0; k < 3; k++) acc += (u128)a[3 * i + k] * a[3 * k + j];
      t[3 * i + j] = (uint64_t)(acc % m);
    }
  std::memcpy(r, t, sizeof t);
}

}  // namespace

void build_mrg_ladder(uint32_t* out) {
  uint64_t A[9] = {0, kMrgA12, kMrgM1 - kMrgA13n, 1, 0, 0, 0, 1, 0};
  uint64_t B[9] = {kMrgA21, 0, kMrgM2 - kMrgA23n, 1, 0, 0, 0, 1, 0};
  for (int b = 0; b < kLadder; b++) {
    for (int i = 0; i < 9; i++) {
      out[b * 18 + i] = (uint32_t)A[i];
      out[b * 18 + 9 + i] = (uint32_t)B[i];
    }
    mat3_sqr(A, A, kMrgM1);
    mat3_sqr(B, B, kMrgM2);
  }
}

namespace {
void mat3_mul(const uint64_t* a, const uint64_t* b, uint64_t* r, uint64_t m) {
  uint64_t t[9];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      u128 acc = 0;
      for (int k = 0; k < 3; k++) acc += (u128)a[3 * i + k] * b[3 * k + j];
      t[3 * i + j] = (uint64_t)(acc % m);
    }
  std::memcpy(r, t, sizeof t);
}
// a^e mod m for a 3x3 matrix
void mat3_pow(const uint64_t* a, uint64_t e, uint64_t* r, uint64_t m) {
  uint64_t p[9], acc[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  std::memcpy(p, a, sizeof p);
  for (; e; e >>= 1) {
    if (e & 1) mat3_mul(acc, p, acc, m);
    mat3_sqr(p, p, m);
  }
  std::memcpy(r, acc, sizeof acc);
}
}  // namespace

void build_mrg_section_table(uint64_t seclen, uint32_t* out) {
  const uint64_t A[9] = {0, kMrgA12, kMrgM1 - kMrgA13n, 1, 0, 0, 0, 1, 0};
  const uint64_t B[9] = {kMrgA21, 0, kMrgM2 - kMrgA23n, 1, 0, 0, 0, 1, 0};
  uint64_t SA[9], SB[9], MA[9], MB[9];
  mat3_pow(A, seclen, SA, kMrgM1);
  mat3_pow(B, seclen, SB, kMrgM2);
  std::memcpy(MA, SA, sizeof MA);
  std::memcpy(MB, SB, sizeof MB);
  for (int j = 1; j < kSectionTableRows + 1; j++) {
    for (int i = 0; i < 9; i++) {
      out[(j - 1) * 18 + i] = (uint32_t)MA[i];
      out[(j - 1) * 18 + 9 + i] = (uint32_t)MB[i];
    }
    mat3_mul(SA, MA, MA, kMrgM1);
    mat3_mul(SB, MB, MB, kMrgM2);
  }
}

// ----------------------------------------------------------------- LFSR113
namespace {
constexpr int kLfP[4] = {31, 29, 28, 25};
constexpr int kLfQ[4] = {6, 2, 13, 3};
constexpr int kLfS[4] = {18, 2, 7, 13};

uint32_t lfsr_word_step(uint32_t z, int c) {
  const uint32_t mask = 0xFFFFFFFFu << (32 - kLfP[c]);
  return ((z & mask) << kLfS[c]) ^ (((z << kLfQ[c]) ^ z) >> (kLfP[c] - kLfS[c]));
}
uint32_t f2_apply(const uint32_t* cols, uint32_t v) {
  uint32_t r = 0;
  while (v) {
    int j = __builtin_ctz(v);
    r ^= cols[j];
    v &= v - 1;
  }
  return r;
}
}  // namespace

void build_lfsr_ladder(uint32_t* out) {
  for (int c = 0; c < 4; c++) {
    uint32_t cols[32];
    for (int j = 0; j < 32; j++) cols[j] = lfsr_word_step(1u << j, c);
    for (int b = 0; b < kLadder; b++) {
      std::memcpy(out + ((size_t)b * 4 + c) * 32, cols, sizeof cols);
      uint32_t sq[32];
      for (int j = 0; j < 32; j++) sq[j] = f2_apply(cols, cols[j]);
      std::memcpy(cols, sq, sizeof sq);
    }
  }
}

// columns of T_c^(d 2^(kLfsrByteE + 8 j)) for every byte position j and
// value d (row [j][d], 128 words, the layout of the section tables)
void build_lfsr_byte_table(uint32_t* out) {
  for (int c = 0; c < 4; c++) {
    uint32_t b[32], t[32], m[32];
    for (int j = 0; j < 32; j++) b[j] = lfsr_word_step(1u << j, c);
    for (int i = 0; i < kLfsrByteE; i++) {   // b = T_c^(2^e)
      for (int j = 0; j < 32; j++) t[j] = f2_apply(b, b[j]);
      std::memcpy(b, t, sizeof t);
    }
    for (int pos = 0; pos < 8; pos++) {
      for (int j = 0; j < 32; j++) m[j] = 1u << j;   // d = 0: identity
      for (int d = 0; d < 256; d++) {
        std::memcpy(out + (((size_t)pos * 256 + d) * 4 + c) * 32, m, sizeof m);
        for (int j = 0; j < 32; j++) t[j] = f2_apply(b, m[j]);
        std::memcpy(m, t, sizeof t);
      }
      for (int i = 0; i < 8; i++) {   // b = b^256 for the next byte
        for (int j = 0; j < 32; j++) t[j] = f2_apply(b, b[j]);
        std::memcpy(b, t, sizeof t);
      }
    }
  }
}

void build_lfsr_section_table(uint64_t seclen, uint32_t* out) {
  for (int c = 0; c < 4; c++) {
    // S = T_c^seclen by squaring; columns of the composition P o Q are P
    // applied to the columns of Q
    uint32_t p[32], s[32], m[32], t[32];
    for (int j = 0; j < 32; j++) {
      p[j] = lfsr_word_step(1u << j, c);
      s[j] = 1u << j;
    }
    for (uint64_t e = seclen; e; e >>= 1) {
      if (e & 1) {
        for (int j = 0; j < 32; j++) t[j] = f2_apply(p, s[j]);
        std::memcpy(s, t, sizeof t);
      }
      for (int j = 0; j < 32; j++) t[j] = f2_apply(p, p[j]);
      std::memcpy(p, t, sizeof t);
    }
    std::memcpy(m, s, sizeof m);
    for (int j = 1; j < kSectionTableRows + 1; j++) {
      std::memcpy(out + ((size_t)(j - 1) * 4 + c) * 32, m, sizeof m);
      for (int i = 0; i < 32; i++) t[i] = f2_apply(s, m[i]);
      std::memcpy(m, t, sizeof t);
    }
  }
}

// ------------------------------------------------------------------- GM/GQ
namespace {
struct Mat2 {
  uint64_t a, b, c, d;
};
Mat2 mat2_mul(const Mat2& x, const Mat2& y, uint64_t p) {
  return Mat2{(uint64_t)(((u128)x.a * y.a + (u128)x.b * y.c) % p), (uint64_t)(((u128)x.a * y.b + (u128)x.b * y.d) % p),
              (uint64_t)(((u128)x.c * y.a + (u128)x.d * y.c) % p), (uint64_t)(((u128)x.c * y.b + (u128)x.d * y.d) % p)};
}
uint64_t pow_mod(uint64_t x, uint64_t e, uint64_t p) {
  uint64_t r = 1 % p;
  for (; e; e >>= 1) {
    if (e & 1) r = (uint64_t)((u128)r * x % p);
    x = (uint64_t)((u128)x * x % p);
  }
  return r;
}
}  // namespace

// out [8][8][256][4]: M^(d 2^(kGmByteE[g] + 8 j)) mod p; neg [8][4]: M^(-n0)
// mod p (the inverse of M^n0 through the adjugate and det^(p-2), p prime),
// the identity where n0 = 0
void build_gm_byte_tables(uint64_t* out, uint64_t* neg) {
  for (int g = 0; g < 8; g++) {
    const GmParams& P = kGmParams[g];
    const uint64_t p = P.p;
    const Mat2 m{P.k % p, (p - P.q % p) % p, 1, 0};
    Mat2 b = m;
    for (int i = 0; i < kGmByteE[g]; i++) b = mat2_mul(b, b, p);
    for (int pos = 0; pos < 8; pos++) {
      Mat2 t{1, 0, 0, 1};
      for (int d = 0; d < 256; d++) {
        uint64_t* o = out + (((size_t)g * 8 + pos) * 256 + d) * 4;
        o[0] = t.a; o[1] = t.b; o[2] = t.c; o[3] = t.d;
        t = mat2_mul(t, b, p);
      }
      for (int i = 0; i < 8; i++) b = mat2_mul(b, b, p);
    }
    Mat2 f{1, 0, 0, 1};
    for (int i = 0; i < P.n0; i++) f = mat2_mul(f, m, p);
    const uint64_t det = (uint64_t)(((u128)f.a * f.d + (u128)(p - f.b) * f.c) % p);
    const uint64_t inv = pow_mod(det, p - 2, p);
    uint64_t* o = neg + (size_t)g * 4;
    o[0] = (uint64_t)((u128)f.d * inv % p);
    o[1] = (uint64_t)((u128)((p - f.b) % p) * inv % p);
    o[2] = (uint64_t)((u128)((p - f.c) % p) * inv % p);
    o[3] = (uint64_t)((u128)f.a * inv % p);
  }
}

void build_gm_ladders(uint64_t* out) {
  for (int g = 0; g < 8; g++) {
    const GmParams& P = kGmParams[g];
    const uint64_t p = P.p;
    uint64_t a = P.k % p, b = (p - P.q % p) % p, c = 1, d = 0;
    for (int i = 0; i < kLadder; i++) {
      uint64_t* o = out + ((size_t)g * kLadder + i) * 4;
      o[0] = a; o[1] = b; o[2] = c; o[3] = d;
      uint64_t na = (uint64_t)(((u128)a * a + (u128)b * c) % p);
      uint64_t nb = (uint64_t)(((u128)a * b + (u128)b * d) % p);
      uint64_t nc = (uint64_t)(((u128)c * a + (u128)d * c) % p);
      uint64_t nd = (uint64_t)(((u128)c * b + (u128)d * d) % p);
      a = na; b = nb; c = nc; d = nd;
    }
  }
}

}  // namespace prand
