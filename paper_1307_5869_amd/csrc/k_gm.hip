// GM19, GM29, GM31, GM55, GM61, GQ58.1, GQ58.3, GQ58.4 on gfx950: ensembles of
// s torus maps x_i^(n) = k x_i^(n-1) - q x_i^(n-2) mod g (paper, equation
// rec1; k, q, g, v of Table 2).  Each element contributes a v-bit digit
// floor(2^v x / g) per step; digits are packed element 0 first, most
// significant bit first, into 32-bit words (GQ58.3: 36 bits per step, 9 words
// per 8 steps).
//
// v = 1 ensembles (s = 32): one lane per element, half a wavefront per
// stream, one ballot per step packs a word; each lane keeps the word of one
// step of every 32, so a flush writes consecutive words from consecutive
// lanes.  GM55, GQ58.3, GQ58.4: one lane per section, every element stepped
// in that lane (dev_gmlane.h); a stream is cut into up to 64 sections that
// start by jumps.
//
// Arithmetic is exact: special-form reductions (2^29-3, 2^31-1, 2^61-1,
// 2^51-129) in integers; GM19 (2^19-1) in FP32 FMAs on centred residues,
// every value an integer below 2^24 (dev_gm.h).  For g = p 2^t (GM55: t = 4, GQ58: t = 29) the even
// k and q kill the 2-adic part within n0 steps; from then on x = 2^t y with y
// following the same recurrence mod p and the digit equal to
// floor(2^v y / p), so the kernels run exact mod-g steps only until every
// element of the wavefront has collapsed and then switch to the mod-p
// recurrence.  In the steady state an element (GM19 aside) is held as a
// redundant residue (congruent to the exact value, possibly shifted by a constant, in
// a range a little wider than the modulus), so no step needs a final
// conditional subtraction; digits are read off that form and states are
// written back exact.
#include "dev_gm.h"
#include "dev_gmlane.h"

namespace prand {
namespace {

using namespace gm;

template <int G, int DT>
__global__ void __launch_bounds__(256) gm_gen32_kernel(const GmState* sin, GmState* sout, uint32_t count, uint64_t n,
                                                       void* __restrict__ out) {
  const uint64_t s = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 5;
  const bool live = s < count;
  constexpr int es = (DT == PRAND_F64) ? 8 : 4;
  gen32_wave<G, DT, false>(live, sin + (live ? s : 0), 0, n, (char*)out + s * n * es, sout + (live ? s : 0), nullptr);
}

// GM55, GQ58.3, GQ58.4: lane gid owns section gid & (nsec - 1) of stream
// gid >> nsec_log2; the sections of a stream cover [j seclen, min((j + 1)
// seclen, n)) and sit in one wavefront (nsec <= 64), so the state read of
// every section precedes the write-back of the last.  Flush width: 64-byte
// runs per lane; GQ58.3 whole 128-byte lines (a 48-word ring, 13 KB per
// wavefront), which measured 4-6 % faster in u32/f32 and 22 % in f64 for
// it and no faster for GM55 and GQ58.4.
template <int G>
constexpr int lane_flush_words() {
  return G == 6 ? 32 : kLaneFlushWide;
}

template <int G, int DT>
__global__ void __launch_bounds__(256) gm_lane_kernel(const GmState* sin, GmState* sout, uint32_t count, uint64_t n,
                                                      int nsec_log2, uint64_t seclen, void* __restrict__ out,
                                                      const uint64_t* __restrict__ ladder) {
  constexpr int FW = lane_flush_words<G>();
  __shared__ __align__(16) uint32_t stage[4][LaneRing<FW>::kWaveWords];
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t nsec = 1ull << nsec_log2;
  const uint64_t jlast = (n == 0) ? 0 : (n - 1) / seclen;
  const uint64_t s = gid >> nsec_log2, j = gid & (nsec - 1);
  const uint64_t start = j * seclen;
  const bool live = s < count && j <= jlast;
  const uint64_t len = live ? ((j == jlast) ? n - start : seclen) : 0;
  constexpr int es = (DT == PRAND_F64) ? 8 : 4;
  void* o = (char*)out + (live ? (s * n + start) * es : 0);
  gmlane_wave<G, DT, true, FW>(stage[threadIdx.x >> 6], live, sin + (live ? s : 0), start, len, o,
                               (live && j == jlast) ? sout + s : nullptr, ladder);
}

// One lane per element slot (32 per stream): states[s] = base (or states[s])
// jumped by the stream's distance; GQ58.3 distances count words.  Block
// splitting with the default block exponent takes the byte tables (at most
// eight matrices per stream), other distances the ladder (one per set bit).
template <int G>
__global__ void __launch_bounds__(256) gm_jump_kernel(GmState* __restrict__ states, uint32_t count,
                                                      const uint64_t* __restrict__ dist, int nlimbs, int per_stream,
                                                      const uint64_t* __restrict__ ids, int block_e,
                                                      const GmState* __restrict__ base,
                                                      const uint64_t* __restrict__ ladder,
                                                      const uint64_t* __restrict__ bytetab,
                                                      const uint64_t* __restrict__ neg) {
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t s = gid >> 5;
  if (s >= count) return;
  const int e = threadIdx.x & 31;
  const GmState* src = base ? base : states + s;
  uint64_t xc = src->xc[e], xp = src->xp[e];
  const uint32_t off = src->off;
  if (ids && bytetab && block_e == kGmByteE[G]) {
    // whole blocks: the offset inside a GQ58.3 block is kept
    if (e < kGmParams[G].s) jump_bytes_elem<G>(xc, xp, ids[s], bytetab, neg);
    GmState* dst = states + s;
    dst->xc[e] = xc;
    dst->xp[e] = xp;
    if (e == 0) { dst->off = (G == 6) ? off : 0; dst->pad = 0; }
    return;
  }
  uint64_t N[kMaxLimbs + 1];
  for (int l = 0; l <= kMaxLimbs; l++) N[l] = 0;
  if (ids) {
    const uint64_t id = ids[s];
    const int q = block_e >> 6, r = block_e & 63;   // block in ensemble steps
    N[q] = id << r;
    if (r) N[q + 1] = id >> (64 - r);
  } else {
    const uint64_t* d = dist + (per_stream ? (size_t)s * nlimbs : 0);
    for (int l = 0; l < nlimbs; l++) N[l] = d[l];
  }
  uint32_t new_off = 0;
  if (G == 6) {
    if (ids) new_off = off;   // whole blocks: the offset inside the block is kept
    else gq3_words_to_steps(N, off, &new_off);
  }
  if (e < kGmParams[G].s) jump_steps_elem<G>(xc, xp, N, ladder);
  GmState* dst = states + s;
  dst->xc[e] = xc;
  dst->xp[e] = xp;
  if (e == 0) { dst->off = new_off; dst->pad = 0; }
}

template <int G, int DT>
hipError_t launch_gen(const uint64_t* ladder, const GmState* sin, GmState* sout, uint32_t count, uint64_t n, void* out,
                      hipStream_t st) {
  if constexpr (G == 3 || G == 6 || G == 7) {
    // enough lanes to fill the chip: up to 64 sections per stream, each at
    // least 64 outputs long; section lengths are multiples of 4 (16-byte
    // aligned starts) and, for GQ58.3, of 9 (every section starts at the
    // same place in the 9-word block as the stream)
    const uint64_t unit = (G == 6) ? 36 : 4;
    int nsec_log2 = 0;
    while (nsec_log2 < 6 && ((uint64_t)count << nsec_log2) < (1ull << 19) && (n >> (nsec_log2 + 1)) >= 64)
      nsec_log2++;
    uint64_t seclen = (n + (1ull << nsec_log2) - 1) >> nsec_log2;
    seclen = (seclen + unit - 1) / unit * unit;
    if (seclen == 0) seclen = unit;
    const uint64_t lanes = (uint64_t)count << nsec_log2;
    const uint32_t blocks = (uint32_t)((lanes + 255) / 256);
    hipLaunchKernelGGL((gm_lane_kernel<G, DT>), dim3(blocks), dim3(256), 0, st, sin, sout, count, n, nsec_log2,
                       seclen, out, ladder);
  } else {
    const uint64_t lanes = (uint64_t)count * 32;
    const uint32_t blocks = (uint32_t)((lanes + 255) / 256);
    hipLaunchKernelGGL((gm_gen32_kernel<G, DT>), dim3(blocks), dim3(256), 0, st, sin, sout, count, n, out);
  }
  return hipGetLastError();
}

template <int G>
hipError_t launch_gen_g(const uint64_t* ladder, int dtype, const GmState* sin, GmState* sout, uint32_t count,
                        uint64_t n, void* out, hipStream_t st) {
  switch (dtype) {
    case PRAND_U32: return launch_gen<G, PRAND_U32>(ladder, sin, sout, count, n, out, st);
    case PRAND_F32: return launch_gen<G, PRAND_F32>(ladder, sin, sout, count, n, out, st);
    default: return launch_gen<G, PRAND_F64>(ladder, sin, sout, count, n, out, st);
  }
}

template <int G>
hipError_t launch_jump_g(const DeviceTables& T, GmState* states, uint32_t count, const JumpSpec& js,
                         const GmState* base, hipStream_t st) {
  const uint64_t lanes = (uint64_t)count * 32;
  const uint32_t blocks = (uint32_t)((lanes + 255) / 256);
  hipLaunchKernelGGL(gm_jump_kernel<G>, dim3(blocks), dim3(256), 0, st, states, count, js.dist, js.nlimbs,
                     js.per_stream, js.ids, js.block_e, base, T.gm,
                     T.gmbyte ? T.gmbyte + (size_t)G * 8 * 256 * 4 : nullptr, T.gmneg ? T.gmneg + (size_t)G * 4 : nullptr);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gm_generate(const DeviceTables& T, int gen, const GmState* sin, GmState* sout, uint32_t count,
                              uint64_t n, int dtype, void* out, hipStream_t st) {
  switch (gen - PRAND_GM19) {
    case 0: return launch_gen_g<0>(T.gm, dtype, sin, sout, count, n, out, st);
    case 1: return launch_gen_g<1>(T.gm, dtype, sin, sout, count, n, out, st);
    case 2: return launch_gen_g<2>(T.gm, dtype, sin, sout, count, n, out, st);
    case 3: return launch_gen_g<3>(T.gm, dtype, sin, sout, count, n, out, st);
    case 4: return launch_gen_g<4>(T.gm, dtype, sin, sout, count, n, out, st);
    case 5: return launch_gen_g<5>(T.gm, dtype, sin, sout, count, n, out, st);
    case 6: return launch_gen_g<6>(T.gm, dtype, sin, sout, count, n, out, st);
    default: return launch_gen_g<7>(T.gm, dtype, sin, sout, count, n, out, st);
  }
}

hipError_t launch_gm_jump(const DeviceTables& T, int gen, GmState* states, uint32_t count, const JumpSpec& js,
                          const GmState* base, hipStream_t st) {
  switch (gen - PRAND_GM19) {
    case 0: return launch_jump_g<0>(T, states, count, js, base, st);
    case 1: return launch_jump_g<1>(T, states, count, js, base, st);
    case 2: return launch_jump_g<2>(T, states, count, js, base, st);
    case 3: return launch_jump_g<3>(T, states, count, js, base, st);
    case 4: return launch_jump_g<4>(T, states, count, js, base, st);
    case 5: return launch_jump_g<5>(T, states, count, js, base, st);
    case 6: return launch_jump_g<6>(T, states, count, js, base, st);
    default: return launch_jump_g<7>(T, states, count, js, base, st);
  }
}

}  // namespace prand
