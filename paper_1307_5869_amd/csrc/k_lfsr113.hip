// LFSR113 on gfx950: four shift-register components x_n = x_{n-p} + x_{n-p+q}
// mod 2 with (p,q,s) = (31,6,18), (29,2,2), (28,13,7), (25,3,13) (paper,
// relations lfsrRel1 and lfsrOutput).  A component's 32-bit word
// (x_{ns}..x_{ns+31}) advances by ((z & top_p) << s) ^ (((z << q) ^ z) >> (p-s)),
// and the output word is the XOR of the four components.  One lane owns a
// (stream, section) pair with the four words in registers; jumps apply the
// 32x32 F2 matrices T_c^(2^b) of the context ladder for each set bit b.
#include "dev_lfsr.h"
#include "regstream.h"

namespace prand {
namespace {

using namespace lfsr;

__global__ void __launch_bounds__(256) lfsr_jump_kernel(LfsrState* __restrict__ states, uint32_t count,
                                                        const uint64_t* __restrict__ dist, int nlimbs,
                                                        int per_stream, const uint64_t* __restrict__ ids,
                                                        int block_e, const LfsrState* __restrict__ base,
                                                        const uint32_t* __restrict__ ladder,
                                                        const uint32_t* __restrict__ bytetab) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  LfsrState st = base ? *base : states[i];
  if (ids && bytetab && block_e == kLfsrByteE) {
    // block splitting with the default block exponent: one byte-table matrix
    // per nonzero byte of the id
    const uint64_t id = ids[i];
    for (int j = 0; j < 8; j++) {
      const uint32_t d = (uint32_t)(id >> (8 * j)) & 255u;
      if (d) LfsrGen::apply(st, bytetab + ((size_t)j * 256 + d) * kLfsrSectionWords);
    }
    states[i] = st;
    return;
  }
  uint64_t limbs[kMaxLimbs];
  int nl;
  if (ids) {
    for (int l = 0; l < kMaxLimbs; l++) limbs[l] = 0;
    const uint64_t id = ids[i];
    const int q = block_e >> 6, r = block_e & 63;
    limbs[q] = id << r;
    if (r && q + 1 < kMaxLimbs) limbs[q + 1] = id >> (64 - r);
    nl = kMaxLimbs;
  } else {
    const uint64_t* d = dist + (per_stream ? (size_t)i * nlimbs : 0);
    for (int l = 0; l < nlimbs; l++) limbs[l] = d[l];
    nl = nlimbs;
  }
  jump_state(ladder, st.z, limbs, nl);
  states[i] = st;
}

}  // namespace

static_assert(LfsrGen::kSectionWords == kLfsrSectionWords, "section-start table row size");

hipError_t launch_lfsr_generate(const DeviceTables& T, const LfsrState* sin, LfsrState* sout, uint32_t count,
                                uint64_t n, int nsec_log2, uint64_t seclen, int dtype, void* out,
                                const uint32_t* sectab, hipStream_t st) {
  return launch_regstream<LfsrGen>(sin, sout, count, n, nsec_log2, seclen, dtype, out, T.lfsr, sectab, st);
}

hipError_t launch_lfsr_jump(const DeviceTables& T, LfsrState* states, uint32_t count, const JumpSpec& js,
                            const LfsrState* base, hipStream_t st) {
  const uint32_t blocks = (count + 255) / 256;
  hipLaunchKernelGGL(lfsr_jump_kernel, dim3(blocks), dim3(256), 0, st, states, count, js.dist, js.nlimbs,
                     js.per_stream, js.ids, js.block_e, base, T.lfsr, T.lfsrbyte);
  return hipGetLastError();
}

}  // namespace prand
