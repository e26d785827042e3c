// MT19937 jump polynomials on the host (context set-up).
//
// The paper's MT19937 jump (section on MT19937 jump-ahead, equation g_v)
// needs g_v = x^v mod phi, phi the characteristic polynomial of the
// generator's F2-linear transition; computing g_v is sequential work, so the
// paper precomputes polynomials for v = 2^n.  Here phi is found by
// Berlekamp-Massey on 2 * 19937 output bits, and products modulo phi use the
// x86 carry-less multiply (Karatsuba over a schoolbook base) with Barrett
// reduction (mu = floor(x^(2n) / phi)), about 0.1 ms per product, so that
// besides the 2^b ladder the context can hold digit tables
// x^(d * 2^(e + position)) mod phi: a stream id then costs one polynomial
// application per nonzero digit instead of one per set bit.
#include "mt_poly.h"

#include <wmmintrin.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>
#include <vector>

namespace prand {
namespace {

constexpr int kN = kMtDeg;
constexpr int kW = 312;   // 64-bit words of a reduced polynomial (19968 bits)

typedef std::vector<uint64_t> Poly;

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

inline int getbit(const uint64_t* a, size_t i) { return (int)((a[i >> 6] >> (i & 63)) & 1u); }
inline void flipbit(uint64_t* a, size_t i) { a[i >> 6] ^= 1ull << (i & 63); }

inline uint64_t bits64_at(const std::vector<uint64_t>& a, size_t pos) {
  size_t w = pos >> 6, r = pos & 63;
  uint64_t lo = w < a.size() ? a[w] >> r : 0;
  uint64_t hi = (r && w + 1 < a.size()) ? a[w + 1] << (64 - r) : 0;
  return lo | hi;
}

// phi (with its x^19937 term) as kW + 1 words; false unless deg phi = 19937
bool find_phi(Poly& phi) {
  const size_t n = 2 * kN + 64;
  const size_t nw = n / 64 + 2;
  std::vector<uint64_t> rev(nw, 0), C(nw, 0), B(nw, 0), T(nw, 0);
  HostMt g(5489u);
  for (size_t i = 0; i < n; i++)
    if (g.next() & 1u) rev[(n - 1 - i) >> 6] |= 1ull << ((n - 1 - i) & 63);
  C[0] = B[0] = 1;
  size_t L = 0, m = 1;
  for (size_t i = 0; i < n; i++) {
    // discrepancy sum_{j<=L} c_j s_{i-j}; s_{i-j} sits at reversed position n-1-i+j
    const size_t off = n - 1 - i;
    uint64_t acc = 0;
    for (size_t w = 0; w <= L / 64; w++) acc ^= C[w] & bits64_at(rev, off + 64 * w);
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
  if (L != (size_t)kN) return false;
  phi.assign(kW + 1, 0);
  for (int i = 0; i <= kN; i++) {
    const size_t j = kN - i;   // phi_i = c_{L-i}
    if (getbit(C.data(), j)) flipbit(phi.data(), i);
  }
  return true;
}

// r[0..na+nb) = a * b in F2[x]
__attribute__((target("pclmul,sse2"))) void clmul(const uint64_t* a, int na, const uint64_t* b, int nb,
                                                  uint64_t* r) {
  std::memset(r, 0, (size_t)(na + nb) * 8);
  for (int i = 0; i < na; i++) {
    if (!a[i]) continue;
    const __m128i A = _mm_set_epi64x(0, (long long)a[i]);
    for (int j = 0; j < nb; j++) {
      if (!b[j]) continue;
      const __m128i P = _mm_clmulepi64_si128(A, _mm_set_epi64x(0, (long long)b[j]), 0x00);
      r[i + j] ^= (uint64_t)_mm_cvtsi128_si64(P);
      r[i + j + 1] ^= (uint64_t)_mm_cvtsi128_si64(_mm_unpackhi_epi64(P, P));
    }
  }
}

// r[0..2n) = a * b for n <= kBase words: every word product added into a
// 128-bit column, then the columns folded into 64-bit words
constexpr int kBase = 24;
__attribute__((target("pclmul,sse2"))) void mul_base(const uint64_t* a, const uint64_t* b, int n, uint64_t* r) {
  __m128i col[2 * kBase];
  for (int k = 0; k < 2 * n; k++) col[k] = _mm_setzero_si128();
  for (int i = 0; i < n; i++) {
    const __m128i A = _mm_set_epi64x(0, (long long)a[i]);
    for (int j = 0; j < n; j++)
      col[i + j] = _mm_xor_si128(col[i + j], _mm_clmulepi64_si128(A, _mm_set_epi64x(0, (long long)b[j]), 0x00));
  }
  uint64_t carry = 0;
  for (int k = 0; k < 2 * n; k++) {
    r[k] = (uint64_t)_mm_cvtsi128_si64(col[k]) ^ carry;
    carry = (uint64_t)_mm_cvtsi128_si64(_mm_unpackhi_epi64(col[k], col[k]));
  }
}

// r[0..2n) = a * b (n words each) by Karatsuba down to mul_base; tmp holds
// at least 8 n words
void kmul(const uint64_t* a, const uint64_t* b, int n, uint64_t* r, uint64_t* tmp) {
  if (n <= kBase) {
    mul_base(a, b, n, r);
    return;
  }
  const int h = (n + 1) / 2, l = n - h;   // a = a0 + x^(64 h) a1, a1 of l <= h words
  uint64_t* sa = tmp;                      // a0 + a1 (h words)
  uint64_t* sb = tmp + h;                  // b0 + b1
  uint64_t* z1 = tmp + 2 * h;              // (a0 + a1)(b0 + b1), 2 h words
  uint64_t* sub = tmp + 4 * h;             // scratch of the recursive calls
  for (int i = 0; i < h; i++) {
    sa[i] = a[i] ^ (i < l ? a[h + i] : 0);
    sb[i] = b[i] ^ (i < l ? b[h + i] : 0);
  }
  kmul(a, b, h, r, sub);                   // z0 -> r[0 .. 2h)
  if (l == h) {
    kmul(a + h, b + h, l, r + 2 * h, sub); // z2 -> r[2h .. 2n)
  } else {
    // odd split: z2 of the shorter halves, padded to h words
    uint64_t* pa = sub;
    uint64_t* pb = sub + h;
    uint64_t* pz = sub + 2 * h;
    for (int i = 0; i < h; i++) {
      pa[i] = i < l ? a[h + i] : 0;
      pb[i] = i < l ? b[h + i] : 0;
    }
    kmul(pa, pb, h, pz, sub + 4 * h);
    for (int i = 0; i < 2 * l; i++) r[2 * h + i] = pz[i];
  }
  kmul(sa, sb, h, z1, sub);
  // middle term z1 - z0 - z2 at word offset h
  for (int i = 0; i < 2 * h; i++) {
    const uint64_t z0 = r[i];
    const uint64_t z2 = i < 2 * l ? r[2 * h + i] : 0;
    z1[i] ^= z0 ^ z2;
  }
  for (int i = 0; i < 2 * h && h + i < 2 * n; i++) r[h + i] ^= z1[i];
}

// a >> s into out (nout words)
void shr(const uint64_t* a, int na, int s, uint64_t* out, int nout) {
  const int q = s >> 6, r = s & 63;
  for (int w = 0; w < nout; w++) {
    const int i = w + q;
    uint64_t lo = i < na ? a[i] >> r : 0;
    uint64_t hi = (r && i + 1 < na) ? a[i + 1] << (64 - r) : 0;
    out[w] = lo | hi;
  }
}

struct Field {
  Poly phi;   // kW + 1 words
  Poly mu;    // floor(x^(2n) / phi), degree n: kW + 1 words

  bool init() {
    if (!find_phi(phi)) return false;
    // long division of x^(2n) by phi
    const int tw = 2 * kW + 2;
    std::vector<uint64_t> rem(tw, 0);
    flipbit(rem.data(), 2 * kN);
    mu.assign(kW + 1, 0);
    for (int d = 2 * kN; d >= kN; d--) {
      if (!getbit(rem.data(), d)) continue;
      flipbit(mu.data(), d - kN);
      const int sh = d - kN, q = sh >> 6, r = sh & 63;
      for (int w = 0; w <= kW; w++) {
        rem[w + q] ^= phi[w] << r;
        if (r && w + q + 1 < tw) rem[w + q + 1] ^= phi[w] >> (64 - r);
      }
    }
    return true;
  }

  // r = a * b mod phi (a, b, r: kW words, degree < n)
  void mulmod(const uint64_t* a, const uint64_t* b, uint64_t* r) const {
    uint64_t c[2 * kW + 2], hi[kW + 1], t[2 * kW + 2], q[kW + 1], s[2 * kW + 2], tmp[8 * (kW + 1)];
    kmul(a, b, kW, c, tmp);                 // degree < 2n - 1
    shr(c, 2 * kW, kN, hi, kW + 1);         // c div x^n
    kmul(hi, mu.data(), kW + 1, t, tmp);
    shr(t, 2 * kW + 2, kN, q, kW + 1);      // quotient
    kmul(q, phi.data(), kW + 1, s, tmp);
    for (int w = 0; w < kW; w++) r[w] = c[w] ^ s[w];
    r[kW - 1] &= (1ull << (kN - 64 * (kW - 1))) - 1;   // keep bits < n
  }
};

void store(const uint64_t* p, uint32_t* out) {
  for (int w = 0; w < kW; w++) {
    out[2 * w] = (uint32_t)p[w];
    out[2 * w + 1] = (uint32_t)(p[w] >> 32);
  }
}

}  // namespace

bool mt_build_polys(uint32_t* ladder, int nladder, uint32_t* dig_lo, uint32_t* dig8hi, int digit_e) {
  Field F;
  if (!F.init()) return false;
  std::vector<uint64_t> lad((size_t)nladder * kW, 0);
  lad[0] = 2;   // x
  for (int b = 0; b + 1 < nladder; b++) F.mulmod(&lad[(size_t)b * kW], &lad[(size_t)b * kW], &lad[(size_t)(b + 1) * kW]);
  for (int b = 0; b < nladder; b++) store(&lad[(size_t)b * kW], ladder + (size_t)b * kMtPolyWords);
  if (!dig_lo && !dig8hi) return true;
  if (digit_e + 64 > nladder) return false;
  // work items: (digit base exponent, digit width, first digit, last digit, output table)
  struct Item {
    int e, width;
    uint32_t d0, d1;
    uint32_t* out;
  };
  std::vector<Item> items;
  if (dig_lo) {
    std::memset(dig_lo, 0, sizeof(uint32_t) * kMtLoDigits * kMtLoSize * kMtPolyWords);
    for (int k = 0; k < kMtLoDigits; k++)
      for (uint32_t d0 = 1; d0 < (uint32_t)kMtLoSize; d0 += 256)
        items.push_back({digit_e + kMtLoBits * k, kMtLoBits, d0, std::min<uint32_t>(d0 + 256, kMtLoSize),
                         dig_lo + (size_t)k * kMtLoSize * kMtPolyWords});
  }
  if (dig8hi) {
    std::memset(dig8hi, 0, sizeof(uint32_t) * 2 * 256 * kMtPolyWords);
    for (int j = 0; j < 2; j++)
      items.push_back({digit_e + 48 + 8 * j, 8, 1, 256, dig8hi + (size_t)j * 256 * kMtPolyWords});
  }
  // x^(d 2^e): the first digit of an item from the ladder (one factor per set
  // bit), each next one by one more multiplication by x^(2^e)
  std::atomic<size_t> next(0);
  auto work = [&]() {
    std::vector<uint64_t> g(kW), nxt(kW);
    for (size_t i; (i = next.fetch_add(1)) < items.size();) {
      const Item& it = items[i];
      const uint64_t* P = &lad[(size_t)it.e * kW];
      bool have = false;
      for (int b = 0; b < it.width; b++) {
        if (!((it.d0 >> b) & 1u)) continue;
        const uint64_t* Q = &lad[(size_t)(it.e + b) * kW];
        if (!have) {
          std::copy(Q, Q + kW, g.begin());
          have = true;
        } else {
          F.mulmod(g.data(), Q, nxt.data());
          g.swap(nxt);
        }
      }
      for (uint32_t d = it.d0; d < it.d1; d++) {
        store(g.data(), it.out + (size_t)d * kMtPolyWords);
        if (d + 1 < it.d1) {
          F.mulmod(g.data(), P, nxt.data());
          g.swap(nxt);
        }
      }
    }
  };
  const unsigned hw = std::thread::hardware_concurrency();
  const unsigned nth = std::max(1u, std::min(16u, hw ? hw : 1u));
  std::vector<std::thread> th;
  for (unsigned t = 1; t < nth; t++) th.emplace_back(work);
  work();
  for (auto& t : th) t.join();
  return true;
}

bool mt_build_block_polys(int nladder, int first, int nblk, uint32_t* blk, uint32_t* inv) {
  if (first + nblk + 9 > nladder) return false;
  Field F;
  if (!F.init()) return false;
  std::vector<uint64_t> lad((size_t)nladder * kW, 0);
  lad[0] = 2;   // x
  for (int b = 0; b + 1 < nladder; b++) F.mulmod(&lad[(size_t)b * kW], &lad[(size_t)b * kW], &lad[(size_t)(b + 1) * kW]);
  // 624 2^k = 2^(k+9) + 2^(k+6) + 2^(k+5) + 2^(k+4)
  std::vector<uint64_t> g(kW), t(kW);
  for (int i = 0; i < nblk; i++) {
    const int k = first + i;
    F.mulmod(&lad[(size_t)(k + 9) * kW], &lad[(size_t)(k + 6) * kW], g.data());
    F.mulmod(g.data(), &lad[(size_t)(k + 5) * kW], t.data());
    F.mulmod(t.data(), &lad[(size_t)(k + 4) * kW], g.data());
    store(g.data(), blk + (size_t)i * kMtPolyWords);
  }
  // (phi - 1) / x: phi's bits 1 .. n moved down one place (degree n - 1)
  std::vector<uint64_t> q(kW, 0);
  if (!(F.phi[0] & 1u)) return false;
  shr(F.phi.data(), kW + 1, 1, q.data(), kW);
  store(q.data(), inv);
  return true;
}

}  // namespace prand

// Host check of the whole-block jump table (not part of the public ABI; the
// test suite compares it with the oracle's x^N mod phi on the CPU): writes
// entry i of the table built for sections of 624 * 2^first outputs, i.e.
// x^(624 * 2^(first + i)) mod phi, and x^(-1) mod phi.  Returns 0, or -1.
extern "C" int prand_internal_mt_block_poly(int first, int i, uint32_t* out624, uint32_t* inv624) {
  if (first < 0 || i < 0 || first + i > 480 || !out624 || !inv624) return -1;
  std::vector<uint32_t> blk((size_t)(i + 1) * prand::kMtPolyWords);
  if (!prand::mt_build_block_polys(first + i + 10, first, i + 1, blk.data(), inv624)) return -1;
  for (int w = 0; w < prand::kMtPolyWords; w++) out624[w] = blk[(size_t)i * prand::kMtPolyWords + w];
  return 0;
}
