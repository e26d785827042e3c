// MRG32K3A on gfx950: X_{n+1} = A X_n mod m1, Y_{n+1} = B Y_n mod m2 (paper,
// section on jumping ahead for MRG32K3A), output z = (x - y) mod m1 in
// [1, m1].  One lane owns one (stream, section) pair and keeps the six state
// words in registers (the store path is shared, see regstream.h).
//
// The recurrence runs in exact double arithmetic on centred residues
// r = p - m * rint(p / m): every product sum is an integer below 2^53 in
// magnitude, rint of the rounded quotient is within one half plus 2^-32 of
// p / m, so |r| <= m/2 + 1 < 2^31 with no correction step, and the next
// step's products (21-bit constants times 31-bit values) stay exact.  A step
// is five FP64 operations per component.  The output map converts the two
// centred values to 32-bit integers and forms the canonical z with integer
// compares and selects (twelve 32-bit operations).
// Jumps apply A^(2^b), B^(2^b) from the context ladder for each set bit b of
// the distance (binary decomposition, O(log n)).
#pragma once

#include "prand_impl.h"

namespace prand {
namespace mrg {


constexpr double kM1 = 4294967087.0;
constexpr double kM2 = 4294944443.0;
constexpr double kInvM1 = 1.0 / 4294967087.0;
constexpr double kInvM2 = 1.0 / 4294944443.0;
constexpr double kNorm = 1.0 / 4294967088.0;   // RN(1/(m1+1))

struct Regs {
  double x0, x1, x2, y0, y1, y2;   // x_n, x_{n-1}, x_{n-2}, ... as centred residues
};

// centred residue of a state word v < 2^32
__device__ __forceinline__ double centre(uint32_t v, double m) {
  const double d = (double)v;
  return d > 0.5 * m ? d - m : d;
}

// p - m * rint(p * (1/m)): a residue of p in [-m/2 - 1, m/2 + 1] for any
// integer |p| < 2^53
__device__ __forceinline__ double reduce_centred(double p, double m, double inv) {
  const double k = __builtin_rint(p * inv);
  return fma(-k, m, p);
}

// canonical residue in [0, m) of a centred one, m = 2^32 - C
template <uint32_t C>
__device__ __forceinline__ uint32_t canonical(double r) {
  const int32_t i = (int32_t)r;                       // exact: |r| < 2^31
  return (uint32_t)(i + __mul24(i >> 31, (int)C));    // i < 0: i + m = i - C (mod 2^32)
}

__device__ __forceinline__ uint32_t step(Regs& r) {
  const double p1 = fma(1403580.0, r.x1, -810728.0 * r.x2);
  const double p2 = fma(527612.0, r.y0, -1370589.0 * r.y2);
  const double x = reduce_centred(p1, kM1, kInvM1);
  const double y = reduce_centred(p2, kM2, kInvM2);
  r.x2 = r.x1; r.x1 = r.x0; r.x0 = x;
  r.y2 = r.y1; r.y1 = r.y0; r.y0 = y;
  const uint32_t xc = canonical<209u>(x), yc = canonical<22853u>(y);
  const uint32_t d = xc - yc;
  return xc > yc ? d : d - 209u;   // x <= y: x - y + m1 = x - y - 209 (mod 2^32), in [1, m1]
}

// 2^32 = C (mod 2^32 - C): fold a 64-bit value to its residue
template <uint32_t C>
__device__ __forceinline__ uint32_t fold32(uint64_t v) {
  v = (v >> 32) * C + (v & 0xFFFFFFFFull);
  v = (v >> 32) * C + (v & 0xFFFFFFFFull);
  v = (v >> 32) * C + (v & 0xFFFFFFFFull);
  const uint64_t m = (1ull << 32) - C;
  return (uint32_t)(v >= m ? v - m : v);
}

template <uint32_t C>
__device__ __forceinline__ void mat3_apply(const uint32_t* M, uint32_t v[3]) {
  const uint64_t m = (1ull << 32) - C;
  uint32_t r[3];
  for (int i = 0; i < 3; i++) {
    uint64_t acc = 0;
    for (int k = 0; k < 3; k++) acc += fold32<C>((uint64_t)M[3 * i + k] * v[k]);
    acc = acc >= m ? acc - m : acc;
    acc = acc >= m ? acc - m : acc;
    r[i] = (uint32_t)acc;
  }
  v[0] = r[0]; v[1] = r[1]; v[2] = r[2];
}

__device__ __forceinline__ void jump_state(const uint32_t* ladder, uint32_t x[3], uint32_t y[3],
                                           const uint64_t* limbs, int nlimbs) {
  for (int l = 0; l < nlimbs; l++) {
    uint64_t w = limbs[l];
    while (w) {
      int b = __builtin_ctzll(w) + 64 * l;
      w &= w - 1;
      const uint32_t* M = ladder + (size_t)b * 18;
      mat3_apply<209u>(M, x);
      mat3_apply<22853u>(M + 9, y);
    }
  }
}

struct MrgGen {
  using State = MrgState;
  using Regs = mrg::Regs;
  __device__ static Regs load(const MrgState& st) {
    return Regs{centre(st.x[0], kM1), centre(st.x[1], kM1), centre(st.x[2], kM1),
                centre(st.y[0], kM2), centre(st.y[1], kM2), centre(st.y[2], kM2)};
  }
  __device__ static MrgState save(const Regs& r) {
    MrgState o;
    o.x[0] = canonical<209u>(r.x0); o.x[1] = canonical<209u>(r.x1); o.x[2] = canonical<209u>(r.x2);
    o.y[0] = canonical<22853u>(r.y0); o.y[1] = canonical<22853u>(r.y1); o.y[2] = canonical<22853u>(r.y2);
    return o;
  }
  __device__ static void jump(MrgState& st, uint64_t d, const uint32_t* ladder) { jump_state(ladder, st.x, st.y, &d, 1); }
  // one jump matrix pair (A^d mod m1, B^d mod m2), 18 words
  static constexpr int kSectionWords = 18;
  __device__ static void apply(MrgState& st, const uint32_t* M) {
    mat3_apply<209u>(M, st.x);
    mat3_apply<22853u>(M + 9, st.y);
  }
  __device__ static uint32_t next(Regs& r) { return step(r); }
  __device__ static double f64(uint32_t z) { return (double)z * kNorm; }
};

}  // namespace mrg
}  // namespace prand
