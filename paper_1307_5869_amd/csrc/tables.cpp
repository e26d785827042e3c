// Context set-up: the jump-ahead tables, computed once on the host when a
// context is created and then uploaded.  The paper computes its MT19937
// jump polynomials on the CPU as well (section on jumping ahead for MT19937:
// the g_v computation is sequential), and uses ladders of powers 2^j for the
// other generators (binary decomposition of the distance).
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

// ------------------------------------------------------------------- GM/GQ
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

// ----------------------------------------------------------------- MT19937
namespace {
constexpr int kDeg = 19937;
constexpr int kPW = 312;          // 64-bit words of a reduced polynomial

struct HostMt {
  uint32_t mt[624];
  int idx;
  explicit HostMt(uint32_t s) {
    mt[0] = s;
    for (int i = 1; i < 624; i++) mt[i] = 1812433253u * (mt[i - 1] ^ (mt[i - 1] >> 30)) + (uint32_t)i;
    idx = 624;
  }
  uint32_t next() {
    if (idx == 624) {
      for (int j = 0; j < 624; j++) {
        uint32_t y = (mt[j] & 0x80000000u) | (mt[j + 1 < 624 ? j + 1 : 0] & 0x7FFFFFFFu);
        mt[j] = mt[j + 397 < 624 ? j + 397 : j + 397 - 624] ^ (y >> 1) ^ ((y & 1u) * 0x9908B0DFu);
      }
      idx = 0;
    }
    uint32_t y = mt[idx++];
    y ^= y >> 11;
    y ^= (y << 7) & 0x9D2C5680u;
    y ^= (y << 15) & 0xEFC60000u;
    return y ^ (y >> 18);
  }
};

inline uint64_t bits64_at(const std::vector<uint64_t>& a, size_t pos) {
  size_t w = pos >> 6, r = pos & 63;
  uint64_t lo = w < a.size() ? a[w] >> r : 0;
  uint64_t hi = (r && w + 1 < a.size()) ? a[w + 1] << (64 - r) : 0;
  return lo | hi;
}

// phi as kPW words (x^19937 implicit); false unless deg phi == 19937
bool mt_phi(std::vector<uint64_t>& phi) {
  const size_t n = 2 * kDeg + 64;
  const size_t nw = n / 64 + 2;
  // reversed sequence: bit (n-1-i) holds s_i = parity bit of output i
  std::vector<uint64_t> rev(nw, 0), C(nw, 0), B(nw, 0), T(nw, 0);
  HostMt g(5489u);
  for (size_t i = 0; i < n; i++)
    if (g.next() & 1u) rev[(n - 1 - i) >> 6] |= 1ull << ((n - 1 - i) & 63);
  C[0] = B[0] = 1;
  size_t L = 0, m = 1;
  for (size_t i = 0; i < n; i++) {
    // d = sum_{j=0..L} c_j s_{i-j};  s_{i-j} sits at reversed position n-1-i+j
    const size_t off = n - 1 - i;
    uint64_t acc = 0;
    for (size_t w = 0; w <= L / 64; w++) acc ^= C[w] & bits64_at(rev, off + 64 * w);
    if (L % 64 != 63) {
      // bits above L in the last word are zero in C already
    }
    if (!(__builtin_popcountll(acc) & 1)) { m++; continue; }
    T = C;
    const size_t q = m >> 6, r = m & 63;
    for (size_t w = 0; w + q < nw; w++) {
      C[w + q] ^= B[w] << r;
      if (r && w + q + 1 < nw) C[w + q + 1] ^= B[w] >> (64 - r);
    }
    if (2 * L <= i) {
      L = i + 1 - L;
      B = T;
      m = 1;
    } else {
      m++;
    }
  }
  if (L != (size_t)kDeg) return false;
  phi.assign(kPW, 0);
  for (int i = 0; i < kDeg; i++) {
    size_t j = kDeg - i;   // phi_i = c_{L-i}
    if ((C[j >> 6] >> (j & 63)) & 1) phi[i >> 6] |= 1ull << (i & 63);
  }
  return true;
}

// r = a^2 mod (x^19937 + phi_low)
void sqr_mod(const std::vector<uint64_t>& phi, const uint64_t* a, uint64_t* r) {
  uint64_t t[2 * kPW + 2];
  std::memset(t, 0, sizeof t);
  for (int w = 0; w < kPW; w++) {
    uint64_t v = a[w];
    for (int h = 0; h < 2; h++) {
      uint32_t x = (uint32_t)(v >> (32 * h));
      uint64_t s = x;   // spread 32 bits to the even positions of 64
      s = (s | (s << 16)) & 0x0000FFFF0000FFFFull;
      s = (s | (s << 8)) & 0x00FF00FF00FF00FFull;
      s = (s | (s << 4)) & 0x0F0F0F0F0F0F0F0Full;
      s = (s | (s << 2)) & 0x3333333333333333ull;
      s = (s | (s << 1)) & 0x5555555555555555ull;
      t[2 * w + h] = s;
    }
  }
  for (int d = 2 * kDeg - 2; d >= kDeg; d--) {
    if (!((t[d >> 6] >> (d & 63)) & 1)) continue;
    t[d >> 6] ^= 1ull << (d & 63);
    const int sh = d - kDeg, q = sh >> 6, rr = sh & 63;
    if (rr == 0) {
      for (int w = 0; w < kPW; w++) t[w + q] ^= phi[w];
    } else {
      for (int w = 0; w < kPW; w++) {
        t[w + q] ^= phi[w] << rr;
        t[w + q + 1] ^= phi[w] >> (64 - rr);
      }
    }
  }
  std::memcpy(r, t, kPW * 8);
}
}  // namespace

bool build_mt_ladder(uint32_t* out) {
  std::vector<uint64_t> phi;
  if (!mt_phi(phi)) return false;
  std::vector<uint64_t> cur(kPW, 0);
  cur[0] = 2;  // x
  for (int b = 0; b < kLadder; b++) {
    uint32_t* o = out + (size_t)b * 624;
    for (int w = 0; w < kPW; w++) {
      o[2 * w] = (uint32_t)cur[w];
      o[2 * w + 1] = (uint32_t)(cur[w] >> 32);
    }
    sqr_mod(phi, cur.data(), cur.data());
  }
  return true;
}

}  // namespace prand
