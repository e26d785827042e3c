// MRG32K3A on gfx950: X_{n+1} = A X_n mod m1, Y_{n+1} = B Y_n mod m2 (paper,
// section on jumping ahead for MRG32K3A), output z = (x - y) mod m1 in
// [1, m1].  One lane owns one (stream, section) pair and keeps the six state
// words in registers (the store path is shared, see regstream.h).  The recurrence runs in exact double arithmetic: every
// product is an integer below 2^53, so fma + floor(p / m) with a +-1
// correction gives the exact residue at full FP64 rate (gfx950 issues FP64
// FMA at the FP32 rate, integer 32x32 multiplies at a quarter of it).
// Jumps apply A^(2^b), B^(2^b) from the context ladder for each set bit b of
// the distance (binary decomposition, O(log n)).
// MRG32K3A device code (see k_mrg32k3a.hip).
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
  double x0, x1, x2, y0, y1, y2;   // x_n, x_{n-1}, x_{n-2}, ...
};

__device__ __forceinline__ double reduce_exact(double p, double m, double inv) {
  double k = floor(p * inv);
  double r = fma(-k, m, p);
  r = (r < 0.0) ? r + m : r;
  r = (r >= m) ? r - m : r;
  return r;
}

__device__ __forceinline__ double step(Regs& r) {
  double p1 = fma(1403580.0, r.x1, -810728.0 * r.x2);
  double p2 = fma(527612.0, r.y0, -1370589.0 * r.y2);
  double x = reduce_exact(p1, kM1, kInvM1);
  double y = reduce_exact(p2, kM2, kInvM2);
  r.x2 = r.x1; r.x1 = r.x0; r.x0 = x;
  r.y2 = r.y1; r.y1 = r.y0; r.y0 = y;
  double z = x - y;
  return (z <= 0.0) ? z + kM1 : z;
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
    return Regs{(double)st.x[0], (double)st.x[1], (double)st.x[2], (double)st.y[0], (double)st.y[1], (double)st.y[2]};
  }
  __device__ static MrgState save(const Regs& r) {
    MrgState o;
    o.x[0] = (uint32_t)r.x0; o.x[1] = (uint32_t)r.x1; o.x[2] = (uint32_t)r.x2;
    o.y[0] = (uint32_t)r.y0; o.y[1] = (uint32_t)r.y1; o.y[2] = (uint32_t)r.y2;
    return o;
  }
  __device__ static void jump(MrgState& st, uint64_t d, const uint32_t* ladder) { jump_state(ladder, st.x, st.y, &d, 1); }
  __device__ static uint32_t next(Regs& r) { return (uint32_t)step(r); }
  __device__ static double f64(uint32_t z) { return (double)z * kNorm; }
};

}  // namespace mrg
}  // namespace prand
