// LFSR113 on gfx950: four shift-register components x_n = x_{n-p} + x_{n-p+q}
// mod 2 with (p,q,s) = (31,6,18), (29,2,2), (28,13,7), (25,3,13) (paper,
// relations lfsrRel1 and lfsrOutput).  A component's 32-bit word
// (x_{ns}..x_{ns+31}) advances by ((z & top_p) << s) ^ (((z << q) ^ z) >> (p-s)),
// and the output word is the XOR of the four components.  One lane owns a
// (stream, section) pair with the four words in registers; jumps apply the
// 32x32 F2 matrices T_c^(2^b) of the context ladder for each set bit b.
// LFSR113 device code (see k_lfsr113.hip).
#pragma once

#include "prand_impl.h"

namespace prand {
namespace lfsr {


// The two halves occupy disjoint bits (the masked part from bit 32 - k + s
// up, the feedback below it), so they join with an OR, and the mask is
// applied after the shift: one three-input op (v_bitop3_b32, truth table
// 0xEA = (src0 & src1) | src2) joins them, five VALU operations per
// component (the compiler's own form of the masked shift takes six).
__device__ __forceinline__ uint32_t comp(uint32_t z, uint32_t mask, int q, int sh1, int s) {
  return __builtin_amdgcn_bitop3_b32(z << s, mask << s, ((z << q) ^ z) >> sh1, 0xEA);
}

struct LfsrRegs {
  uint32_t z0, z1, z2, z3;
};

__device__ __forceinline__ uint32_t step(LfsrRegs& r) {
  r.z0 = comp(r.z0, 0xFFFFFFFEu, 6, 13, 18);
  r.z1 = comp(r.z1, 0xFFFFFFF8u, 2, 27, 2);
  r.z2 = comp(r.z2, 0xFFFFFFF0u, 13, 21, 7);
  r.z3 = comp(r.z3, 0xFFFFFF80u, 3, 12, 13);
  return __builtin_amdgcn_bitop3_b32(r.z0, r.z1, r.z2, 0x96) ^ r.z3;   // 0x96: three-input XOR
}

__device__ __forceinline__ uint32_t f2_apply(const uint32_t* __restrict__ cols, uint32_t v) {
  uint32_t r = 0;
#pragma unroll 4
  for (int j = 0; j < 32; j++) r ^= ((v >> j) & 1u) ? cols[j] : 0u;
  return r;
}

__device__ __forceinline__ void jump_state(const uint32_t* ladder, uint32_t z[4], const uint64_t* limbs,
                                           int nlimbs) {
  for (int l = 0; l < nlimbs; l++) {
    uint64_t w = limbs[l];
    while (w) {
      const int b = __builtin_ctzll(w) + 64 * l;
      w &= w - 1;
      const uint32_t* M = ladder + (size_t)b * 128;
      for (int c = 0; c < 4; c++) z[c] = f2_apply(M + 32 * c, z[c]);
    }
  }
}

struct LfsrGen {
  using State = LfsrState;
  using Regs = lfsr::LfsrRegs;
  __device__ static Regs load(const LfsrState& st) { return Regs{st.z[0], st.z[1], st.z[2], st.z[3]}; }
  __device__ static LfsrState save(const Regs& r) {
    LfsrState o;
    o.z[0] = r.z0; o.z[1] = r.z1; o.z[2] = r.z2; o.z[3] = r.z3;
    return o;
  }
  __device__ static void jump(LfsrState& st, uint64_t d, const uint32_t* ladder) { jump_state(ladder, st.z, &d, 1); }
  // one jump matrix per component (columns of T_c^d), 4 x 32 words, 16-byte
  // aligned: the columns come in as 16-byte loads, and column j joins the
  // result through bit j of the word spread to a mask (one sign-extending
  // bit-field extract) and one three-input op r ^ (mask & column)
  static constexpr int kSectionWords = 128;
  __device__ static void apply(LfsrState& st, const uint32_t* M) {
    const uint4* m4 = (const uint4*)M;
#pragma unroll
    for (int c = 0; c < 4; c++) {
      const uint32_t v = st.z[c];
      uint32_t r = 0;
#pragma unroll
      for (int q = 0; q < 8; q++) {
        const uint4 col = m4[c * 8 + q];
        const uint32_t cw[4] = {col.x, col.y, col.z, col.w};
#pragma unroll
        for (int t = 0; t < 4; t++) {
          const int j = 4 * q + t;
          const uint32_t mask = (uint32_t)((int32_t)(v << (31 - j)) >> 31);
          r = __builtin_amdgcn_bitop3_b32(r, mask, cw[t], 0x78);
        }
      }
      st.z[c] = r;
    }
  }
  __device__ static uint32_t next(Regs& r) { return step(r); }
  __device__ static double f64(uint32_t w) { return (double)w * 0x1p-32; }
};

}  // namespace lfsr
}  // namespace prand
