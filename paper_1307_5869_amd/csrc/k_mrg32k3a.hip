// MRG32K3A on gfx950: X_{n+1} = A X_n mod m1, Y_{n+1} = B Y_n mod m2 (paper,
// section on jumping ahead for MRG32K3A), output z = (x - y) mod m1 in
// [1, m1].  One lane owns one (stream, section) pair and keeps the six state
// words in registers (the store path is shared, see regstream.h); the
// recurrence runs in exact double arithmetic on centred residues (dev_mrg.h).
// Jumps apply A^(2^b), B^(2^b) from the context ladder for each set bit b of
// the distance (binary decomposition, O(log n)); the sections of the
// many-stream kernel start from one application of a section-start table.
#include "dev_mrg.h"
#include "regstream.h"

namespace prand {
namespace {

using namespace mrg;

// One lane per stream: states[i] = (base ? *base : states[i]) jumped by the
// stream's distance (explicit limbs, or id * 2^block_e).
__global__ void __launch_bounds__(256) mrg_jump_kernel(MrgState* __restrict__ states, uint32_t count,
                                                       const uint64_t* __restrict__ dist, int nlimbs,
                                                       int per_stream, const uint64_t* __restrict__ ids,
                                                       int block_e, const MrgState* __restrict__ base,
                                                       const uint32_t* __restrict__ ladder) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  MrgState st = base ? *base : states[i];
  uint64_t limbs[kMaxLimbs];
  int nl;
  if (ids) {
    // id * 2^block_e as limbs
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
  jump_state(ladder, st.x, st.y, limbs, nl);
  states[i] = st;
}

}  // namespace

static_assert(MrgGen::kSectionWords == kMrgSectionWords, "section-start table row size");

hipError_t launch_mrg_generate(const DeviceTables& T, const MrgState* sin, MrgState* sout, uint32_t count,
                               uint64_t n, int nsec_log2, uint64_t seclen, int dtype, void* out,
                               const uint32_t* sectab, hipStream_t st) {
  return launch_regstream<MrgGen>(sin, sout, count, n, nsec_log2, seclen, dtype, out, T.mrg, sectab, st);
}

hipError_t launch_mrg_jump(const DeviceTables& T, MrgState* states, uint32_t count, const JumpSpec& js,
                           const MrgState* base, hipStream_t st) {
  const uint32_t blocks = (count + 255) / 256;
  hipLaunchKernelGGL(mrg_jump_kernel, dim3(blocks), dim3(256), 0, st, states, count, js.dist, js.nlimbs,
                     js.per_stream, js.ids, js.block_e, base, T.mrg);
  return hipGetLastError();
}

}  // namespace prand
