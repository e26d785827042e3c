// Batched persistent generation: many tasks (generator, state, length,
// dtype, output) of uneven sizes in one launch.
//
// The host cuts every task into tiles, one tile being the work of one
// wavefront: 64 lane-sections of a MRG32K3A / LFSR113 task, 2 / 8 / 4
// element-group sections of a GM/GQ task (32, 8 or 16 lanes per section), or
// a whole MT19937 task (one wavefront per stream).  Sections start from the
// task's state jumped to their first output, so tiles are independent.  A
// fixed grid of wavefronts pulls tile indices from an atomic counter until
// the list is exhausted -- every wavefront reaches that exit -- and runs the
// generator family's wavefront routine, the same code the one-generator
// kernels use.  The tile list is ordered longest first.
#include "dev_gm.h"
#include "dev_lfsr.h"
#include "dev_mrg.h"
#include "dev_mt.h"
#include "prand_batch.h"
#include "regstream.h"

namespace prand {
namespace {

constexpr int kBatchCW = 32;

// Each family's tile routine is kept out of line so that the fused kernel
// needs the registers of the largest routine, not of all of them inlined
// together.

// section geometry of a tile: group gi of the wavefront takes section first + gi
struct Sect {
  bool live;
  uint64_t start, len;
  bool last;
};
__device__ __forceinline__ Sect section_of(const BatchTile& tl, const BatchTask& tk, int groups) {
  const int gi = (threadIdx.x & 63) / (64 / groups);
  Sect s;
  s.live = (uint32_t)gi < tl.nsec;
  s.start = (tl.first + (uint64_t)gi) * tl.seclen;
  s.len = s.live ? (s.start + tl.seclen <= tk.n ? tl.seclen : tk.n - s.start) : 0;
  s.last = s.live && s.start + s.len == tk.n;
  return s;
}

template <int DT>
__device__ __noinline__ void run_mt(const BatchTask& tk, uint32_t* lds) {
  mt::gen_wave<DT>(lds, (const MtState*)tk.state_in, (MtState*)tk.state_out, tk.n, tk.out);
}

template <class G, int DT>
__device__ __noinline__ void run_reg(const BatchTile& tl, const BatchTask& tk, uint32_t* lds, const uint32_t* ladder) {
  constexpr int es = (DT == PRAND_F64) ? 8 : 4;
  const Sect s = section_of(tl, tk, 64);
  void* o = (char*)tk.out + (s.live ? s.start : 0) * es;
  regstream_wave<G, DT, kBatchCW>(lds, s.live, (const typename G::State*)tk.state_in, s.start, s.len, o,
                                  s.last ? (typename G::State*)tk.state_out : nullptr, tl.coalesce != 0, ladder);
}

// GM/GQ: a dead group follows along without loads or stores; the planner
// gives both halves of a v = 1 tile the same length (tl.len32)
template <int G, int DT>
__device__ __noinline__ void run_gm(const BatchTile& tl, const BatchTask& tk, const uint64_t* ladder) {
  constexpr int es = (DT == PRAND_F64) ? 8 : 4;
  constexpr int groups = (G == 3 || G == 7) ? 8 : (G == 6 ? 4 : 2);
  const Sect s = section_of(tl, tk, groups);
  void* o = (char*)tk.out + (s.live ? s.start : 0) * es;
  const GmState* in = (const GmState*)tk.state_in;
  GmState* sout = s.last ? (GmState*)tk.state_out : nullptr;
  if constexpr (G == 6) gm::gq3_wave<DT>(s.live, in, s.start, s.len, o, sout, ladder);
  else if constexpr (groups == 8) gm::gen8_wave<G, DT>(s.live, in, s.start, s.len, o, sout, ladder);
  else gm::gen32_wave<G, DT>(s.live, in, s.start, tl.len32, o, sout, ladder);
}

template <int DT>
__device__ __forceinline__ void run_tile_dt(const BatchTile& tl, const BatchTask& tk, uint32_t* lds,
                                            const DeviceTables& T) {
  switch (tk.gen) {
    case PRAND_MT19937: run_mt<DT>(tk, lds); break;
    case PRAND_MRG32K3A: run_reg<mrg::MrgGen, DT>(tl, tk, lds, T.mrg); break;
    case PRAND_LFSR113: run_reg<lfsr::LfsrGen, DT>(tl, tk, lds, T.lfsr); break;
    case PRAND_GM19: run_gm<0, DT>(tl, tk, T.gm); break;
    case PRAND_GM29: run_gm<1, DT>(tl, tk, T.gm); break;
    case PRAND_GM31: run_gm<2, DT>(tl, tk, T.gm); break;
    case PRAND_GM55: run_gm<3, DT>(tl, tk, T.gm); break;
    case PRAND_GM61: run_gm<4, DT>(tl, tk, T.gm); break;
    case PRAND_GQ58X1: run_gm<5, DT>(tl, tk, T.gm); break;
    case PRAND_GQ58X3: run_gm<6, DT>(tl, tk, T.gm); break;
    default: run_gm<7, DT>(tl, tk, T.gm); break;
  }
}

__global__ void batch_reset_kernel(uint32_t* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

__global__ void __launch_bounds__(256) batch_kernel(const BatchTile* __restrict__ tiles, uint32_t ntiles,
                                                    const BatchTask* __restrict__ tasks, uint32_t* counter,
                                                    DeviceTables T) {
  __shared__ __align__(16) uint32_t lds[4][RegStage<kBatchCW>::kWaveWords];
  uint32_t* mine = lds[threadIdx.x >> 6];
  const int lane = threadIdx.x & 63;
  for (;;) {
    uint32_t t = 0;
    if (lane == 0) t = atomicAdd(counter, 1u);
    t = __builtin_amdgcn_readfirstlane(__shfl(t, 0));
    if (t >= ntiles) break;
    const BatchTile tl = tiles[t];
    const BatchTask tk = tasks[tl.task];
    if (tl.kind == kTileCopy) {
      // n = 0: the output state is the input state
      const uint32_t* a = (const uint32_t*)tk.state_in;
      uint32_t* b = (uint32_t*)tk.state_out;
      for (uint32_t i = lane; i < tl.len32; i += 64) b[i] = a[i];
      continue;
    }
    switch (tk.dtype) {
      case PRAND_U32: run_tile_dt<PRAND_U32>(tl, tk, mine, T); break;
      case PRAND_F32: run_tile_dt<PRAND_F32>(tl, tk, mine, T); break;
      default: run_tile_dt<PRAND_F64>(tl, tk, mine, T); break;
    }
  }
}

}  // namespace

hipError_t launch_batch(const DeviceTables& T, const BatchTile* tiles, uint32_t ntiles, const BatchTask* tasks,
                        uint32_t* counter, uint32_t blocks, hipStream_t st) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, st, counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(batch_kernel, dim3(blocks), dim3(256), 0, st, tiles, ntiles, tasks, counter, T);
  return hipGetLastError();
}

}  // namespace prand
