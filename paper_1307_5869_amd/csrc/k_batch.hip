// Batched generation: many tasks (generator, state, length, dtype, output) of
// uneven sizes in one launch.
//
// The host cuts every task into tiles, one tile being the work of one
// wavefront: 64 lane-sections of a MRG32K3A / LFSR113 / GM55 / GQ58.3 /
// GQ58.4 task, 2 element-group sections of a v = 1 GM/GQ task (32 lanes per
// section), or a whole MT19937 task (one wavefront per stream).  Sections are independent:
// each starts from the task's state jumped to its first output.
//
// A batched launch (prand_batch_launch) is a chain of kernels on one stream:
//  - batch_reset_kernel clears the tile counters;
//  - batch_starts_kernel jumps every MRG32K3A/LFSR113/GM/GQ section to its
//    start and writes the state to the batch's scratch area (the jump code
//    needs many registers, so it runs apart from the generation loops);
//    sections of MT19937 tasks above 2^24 outputs get theirs from
//    mt_section_start_kernel (k_mt19937.hip);
//  - three persistent kernels, one per register class, each launched with
//    as many wavefronts as the chip holds at once: every wavefront takes the
//    next tile of its class's list from a device counter until the list is
//    used up.  The lists are ordered longest first by the host (estimated
//    wavefront time), so the long tiles start at once and the short ones
//    fill the end.  batch_heavy_kernel runs the lane-per-section ensembles
//    (GM55, GQ58.3, GQ58.4), batch_reg_persistent_kernel MRG32K3A/LFSR113
//    (its LDS sized by the chunk width of the staging, the footprint the
//    autotuner chooses), batch_light_kernel MT19937 tasks and sections, the
//    v = 1 GM/GQ tiles and n = 0 copies.  Kept apart, each runs at its own
//    register count: one loop over every family holds the union of their
//    live values (over 100 VGPRs) and halves the resident wavefronts.
// Each tile runs the same wavefront routines as the one-generator kernels.
//
// The serving loop keeps one grid kernel per family (batch_reg_kernel,
// batch_gm_kernel<shape>, batch_mt_v1_kernel) on its iteration stream: its
// iterations are small, and their length is set by the longest chunk.
#include <algorithm>

#include "dev_gm.h"
#include "dev_gmlane.h"
#include "dev_lfsr.h"
#include "dev_mrg.h"
#include "dev_mt.h"
#include "prand_batch.h"
#include "regstream.h"

namespace prand {
namespace {

constexpr int kBatchCW = 32;   // MRG32K3A/LFSR113 staging chunk of the grid kernels

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

constexpr int gm_groups(int G) { return (G == 3 || G == 6 || G == 7) ? 64 : 2; }

// the tile index of this wavefront, known to the compiler as uniform across
// it, so the tile and task fields it loads live in scalar registers
__device__ __forceinline__ uint32_t wave_index() {
  return __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
}

// ---------------------------------------------------------------- starts
template <class G>
__device__ __noinline__ void start_reg(const BatchTile& tl, const BatchTask& tk, char* scratch,
                                       const uint32_t* ladder) {
  const Sect s = section_of(tl, tk, 64);
  if (!s.live) return;
  typename G::State st = *(const typename G::State*)tk.state_in;
  if (s.start) G::jump(st, s.start, ladder);
  ((typename G::State*)(scratch + tl.starts))[threadIdx.x & 63] = st;
}

template <int G>
__device__ __noinline__ void start_gm(const BatchTile& tl, const BatchTask& tk, char* scratch,
                                      const uint64_t* ladder) {
  constexpr int groups = gm_groups(G);
  const Sect s = section_of(tl, tk, groups);
  if (!s.live) return;
  const int lane = threadIdx.x & 63;
  if constexpr (groups == 64) {
    // one lane per section: every element of the section's start state; a
    // jump past n0 steps runs in the fast (mod p) representation
    using E = gm::Eng<G>;
    const GmState* in = (const GmState*)tk.state_in;
    GmState* dst = (GmState*)(scratch + tl.starts) + lane;
    constexpr int S = (G == 6) ? 12 : 8;
    uint64_t nsteps = s.start;
    uint32_t off = (G == 6) ? in->off : 0;
    if (G == 6 && s.start) {   // words from the block start -> whole blocks of 8 steps
      const uint64_t w = (uint64_t)off + s.start;
      nsteps = 8 * (w / 9);
      off = (uint32_t)(w % 9);
    }
    for (int e = 0; e < S; e++) {
      uint64_t xc = in->xc[e], xp = in->xp[e];
      if (nsteps >= (uint64_t)kGmParams[G].n0 || (nsteps && E::collapsed(xc) && E::collapsed(xp))) {
        const gm::FastPair<G> j = gm::lane_jump_fast<G>(in, e, nsteps, ladder);
        xc = E::from_fast(j.yc);
        xp = E::from_fast(j.yp);
      } else if (nsteps) {
        for (uint64_t i = 0; i < nsteps; i++) {
          const uint64_t nx = E::slow_step(xc, xp);
          xp = xc;
          xc = nx;
        }
      }
      dst->xc[e] = xc;
      dst->xp[e] = xp;
    }
    dst->off = off;
    dst->pad = 0;
  } else {
    const int gi = lane / (64 / groups);
    const int e = 31 - (lane & 31);
    uint64_t xc, xp;
    const uint32_t off = gm::load_at<G>((const GmState*)tk.state_in, e, s.start, xc, xp, ladder);
    GmState* dst = (GmState*)(scratch + tl.starts) + gi;
    dst->xc[e] = xc;
    dst->xp[e] = xp;
    if (e == 0) {
      dst->off = off;
      dst->pad = 0;
    }
  }
}

__global__ void __launch_bounds__(256) batch_starts_kernel(const BatchTile* __restrict__ tiles, uint32_t ntiles,
                                                           const BatchTask* __restrict__ tasks, char* scratch,
                                                           DeviceTables T) {
  const uint32_t t = wave_index();
  if (t >= ntiles) return;
  const BatchTile tl = tiles[t];
  const BatchTask tk = tasks[tl.task];
  switch (tk.gen) {
    case PRAND_MRG32K3A: start_reg<mrg::MrgGen>(tl, tk, scratch, T.mrg); break;
    case PRAND_LFSR113: start_reg<lfsr::LfsrGen>(tl, tk, scratch, T.lfsr); break;
    case PRAND_GM19: start_gm<0>(tl, tk, scratch, T.gm); break;
    case PRAND_GM29: start_gm<1>(tl, tk, scratch, T.gm); break;
    case PRAND_GM31: start_gm<2>(tl, tk, scratch, T.gm); break;
    case PRAND_GM55: start_gm<3>(tl, tk, scratch, T.gm); break;
    case PRAND_GM61: start_gm<4>(tl, tk, scratch, T.gm); break;
    case PRAND_GQ58X1: start_gm<5>(tl, tk, scratch, T.gm); break;
    case PRAND_GQ58X3: start_gm<6>(tl, tk, scratch, T.gm); break;
    case PRAND_GQ58X4: start_gm<7>(tl, tk, scratch, T.gm); break;
    default: break;
  }
}

// ------------------------------------------------------- MRG32K3A/LFSR113
template <class G, int DT, int CW = kBatchCW>
__device__ __forceinline__ void gen_reg(const BatchTile& tl, const BatchTask& tk, uint32_t* lds,
                                        const char* scratch) {
  constexpr int es = (DT == PRAND_F64) ? 8 : 4;
  const Sect s = section_of(tl, tk, 64);
  void* o = (char*)tk.out + (s.live ? s.start : 0) * es;
  const typename G::State* in = (const typename G::State*)(scratch + tl.starts) + (threadIdx.x & 63);
  regstream_wave<G, DT, CW, false>(lds, s.live, in, 0, s.len, o,
                                         s.last ? (typename G::State*)tk.state_out : nullptr, tl.coalesce != 0,
                                         nullptr);
}

__global__ void __launch_bounds__(256) batch_reg_kernel(const BatchTile* __restrict__ tiles, uint32_t ntiles,
                                                        const BatchTask* __restrict__ tasks, const char* scratch) {
  __shared__ __align__(16) uint32_t lds[4][RegStage<kBatchCW>::kWaveWords];
  const uint32_t t = wave_index();
  if (t >= ntiles) return;
  uint32_t* mine = lds[(threadIdx.x >> 6) & 3];
  const BatchTile tl = tiles[t];
  const BatchTask tk = tasks[tl.task];
  const bool mrg = tk.gen == PRAND_MRG32K3A;
  switch (tk.dtype) {
    case PRAND_U32:
      if (mrg) gen_reg<mrg::MrgGen, PRAND_U32>(tl, tk, mine, scratch);
      else gen_reg<lfsr::LfsrGen, PRAND_U32>(tl, tk, mine, scratch);
      break;
    case PRAND_F32:
      if (mrg) gen_reg<mrg::MrgGen, PRAND_F32>(tl, tk, mine, scratch);
      else gen_reg<lfsr::LfsrGen, PRAND_F32>(tl, tk, mine, scratch);
      break;
    default:
      if (mrg) gen_reg<mrg::MrgGen, PRAND_F64>(tl, tk, mine, scratch);
      else gen_reg<lfsr::LfsrGen, PRAND_F64>(tl, tk, mine, scratch);
      break;
  }
}

// ------------------------------------------------------------------ GM/GQ
// A dead group follows along without loads or stores; the planner gives both
// halves of a v = 1 tile the same length (tl.len32).
template <int G, int DT>
__device__ __forceinline__ void gen_gm(const BatchTile& tl, const BatchTask& tk, const char* scratch,
                                       uint32_t* rows) {
  constexpr int es = (DT == PRAND_F64) ? 8 : 4;
  constexpr int groups = gm_groups(G);
  const Sect s = section_of(tl, tk, groups);
  void* o = (char*)tk.out + (s.live ? s.start : 0) * es;
  const int gi = (threadIdx.x & 63) / (64 / groups);
  const GmState* in = (const GmState*)(scratch + tl.starts) + (s.live ? gi : 0);
  GmState* sout = s.last ? (GmState*)tk.state_out : nullptr;
  if constexpr (groups == 64)
    gm::gmlane_wave<G, DT, false, gm::kLaneFlushNarrow>(rows, s.live, in, 0, s.len, o, sout, nullptr);
  else gm::gen32_wave<G, DT, false>(s.live, in, 0, tl.len32, o, sout, nullptr);
}

// per ensemble shape, so each kernel runs at its own register count: S = 0:
// v = 1 (32 lanes per section; batch_mt_v1_kernel), 1: v = 4 (a lane per
// section), 2: GQ58.3 (a lane per section)
template <int S, int DT>
__device__ __forceinline__ void gen_gm_dt(const BatchTile& tl, const BatchTask& tk, const char* scratch,
                                          uint32_t* rows) {
  if constexpr (S == 0) {
    switch (tk.gen) {
      case PRAND_GM19: gen_gm<0, DT>(tl, tk, scratch, rows); break;
      case PRAND_GM29: gen_gm<1, DT>(tl, tk, scratch, rows); break;
      case PRAND_GM31: gen_gm<2, DT>(tl, tk, scratch, rows); break;
      case PRAND_GM61: gen_gm<4, DT>(tl, tk, scratch, rows); break;
      default: gen_gm<5, DT>(tl, tk, scratch, rows); break;
    }
  } else if constexpr (S == 1) {
    if (tk.gen == PRAND_GM55) gen_gm<3, DT>(tl, tk, scratch, rows);
    else gen_gm<7, DT>(tl, tk, scratch, rows);
  } else {
    gen_gm<6, DT>(tl, tk, scratch, rows);
  }
}

template <int S>
__global__ void __launch_bounds__(256) batch_gm_kernel(const BatchTile* __restrict__ tiles, uint32_t ntiles,
                                                       const BatchTask* __restrict__ tasks, const char* scratch) {
  static_assert(S == 1 || S == 2, "lane-per-section shapes only");
  __shared__ __align__(16) uint32_t lds[4][gm::LaneRing<gm::kLaneFlushNarrow>::kWaveWords];
  const uint32_t t = wave_index();
  if (t >= ntiles) return;
  uint32_t* rows = lds[(threadIdx.x >> 6) & 3];
  const BatchTile tl = tiles[t];
  const BatchTask tk = tasks[tl.task];
  switch (tk.dtype) {
    case PRAND_U32: gen_gm_dt<S, PRAND_U32>(tl, tk, scratch, rows); break;
    case PRAND_F32: gen_gm_dt<S, PRAND_F32>(tl, tk, scratch, rows); break;
    default: gen_gm_dt<S, PRAND_F64>(tl, tk, scratch, rows); break;
  }
}

// --------------------------------------------------- MT19937 and n = 0 tasks
// A whole MT19937 task, or one kMtSection-output section of a long one: the
// section starts from its state in the scratch; a section that is not the
// task's last leaves its end state in that same slot (read by this
// wavefront only, before it is written).
__device__ __forceinline__ void mt_tile(const BatchTile& tl, const BatchTask& tk, char* scratch, uint32_t* mine) {
  const int lane = threadIdx.x & 63;
  if (tl.kind == kTileCopy) {
    // n = 0: the output state is the input state
    const uint32_t* a = (const uint32_t*)tk.state_in;
    uint32_t* b = (uint32_t*)tk.state_out;
    for (uint32_t i = lane; i < tl.len32; i += 64) b[i] = a[i];
    return;
  }
  const MtState* in = (const MtState*)tk.state_in;
  MtState* out = (MtState*)tk.state_out;
  uint64_t n = tk.n, start = 0;
  if (tl.kind == kTileMtSection) {
    MtState* slot = (MtState*)(scratch + tl.starts);
    start = tl.first * tl.seclen;
    n = (tk.n - start < tl.seclen) ? tk.n - start : tl.seclen;
    in = slot;
    if (start + n < tk.n) out = slot;
  }
  switch (tk.dtype) {
    case PRAND_U32: mt::gen_wave<PRAND_U32>(mine, in, out, n, (char*)tk.out + start * 4); break;
    case PRAND_F32: mt::gen_wave<PRAND_F32>(mine, in, out, n, (char*)tk.out + start * 4); break;
    default: mt::gen_wave<PRAND_F64>(mine, in, out, n, (char*)tk.out + start * 8); break;
  }
}

// wavefronts 0 .. nmt-1 take the MT19937 tiles, the next nv1 the v = 1 GM/GQ
// tiles (the branch is uniform per wavefront)
__global__ void __launch_bounds__(256) batch_mt_v1_kernel(const BatchTile* __restrict__ mt_tiles, uint32_t nmt,
                                                          const BatchTile* __restrict__ v1_tiles, uint32_t nv1,
                                                          const BatchTask* __restrict__ tasks, char* scratch) {
  __shared__ __align__(16) uint32_t mt[4][624];
  const uint32_t t = wave_index();
  if (t < nmt) {
    const BatchTile tl = mt_tiles[t];
    mt_tile(tl, tasks[tl.task], scratch, mt[(threadIdx.x >> 6) & 3]);
    return;
  }
  if (t - nmt >= nv1) return;
  const BatchTile tl = v1_tiles[t - nmt];
  const BatchTask tk = tasks[tl.task];
  switch (tk.dtype) {
    case PRAND_U32: gen_gm_dt<0, PRAND_U32>(tl, tk, scratch, nullptr); break;
    case PRAND_F32: gen_gm_dt<0, PRAND_F32>(tl, tk, scratch, nullptr); break;
    default: gen_gm_dt<0, PRAND_F64>(tl, tk, scratch, nullptr); break;
  }
}

// ---------------------------------------------------------- persistent
__global__ void batch_reset_kernel(uint32_t* counters) {
  if (threadIdx.x < kBatchCounters) counters[threadIdx.x] = 0;
}

// the next entry of a tile list for this wavefront (uniform across it)
__device__ __forceinline__ uint32_t next_tile(uint32_t* counter) {
  uint32_t k = 0;
  if ((threadIdx.x & 63) == 0) k = atomicAdd(counter, 1u);
  return __builtin_amdgcn_readfirstlane(__shfl(k, 0));
}

template <int CW>
struct RegLds {
  static constexpr int kWords = RegStage<CW>::kWaveWords;
};

// MT19937 tasks and sections, v = 1 GM/GQ tiles and n = 0 copies
__global__ void __launch_bounds__(256) batch_light_kernel(const BatchTile* __restrict__ tiles,
                                                          const uint32_t* __restrict__ order, uint32_t n,
                                                          const BatchTask* __restrict__ tasks, char* scratch,
                                                          uint32_t* counter) {
  __shared__ __align__(16) uint32_t mt[4][624];
  uint32_t* mine = mt[(threadIdx.x >> 6) & 3];
  for (;;) {
    const uint32_t k = next_tile(counter);
    if (k >= n) break;
    const BatchTile tl = tiles[order[k]];
    const BatchTask tk = tasks[tl.task];
    if (tk.gen == PRAND_MT19937 || tl.kind == kTileCopy) {
      mt_tile(tl, tk, scratch, mine);
    } else {
      switch (tk.dtype) {
        case PRAND_U32: gen_gm_dt<0, PRAND_U32>(tl, tk, scratch, nullptr); break;
        case PRAND_F32: gen_gm_dt<0, PRAND_F32>(tl, tk, scratch, nullptr); break;
        default: gen_gm_dt<0, PRAND_F64>(tl, tk, scratch, nullptr); break;
      }
    }
    wave_lds_sync();   // the next tile reuses this wavefront's LDS
  }
}

// MRG32K3A/LFSR113 tiles, LDS staging chunks of CW words
template <int CW>
__global__ void __launch_bounds__(256) batch_reg_persistent_kernel(const BatchTile* __restrict__ tiles,
                                                                   const uint32_t* __restrict__ order, uint32_t n,
                                                                   const BatchTask* __restrict__ tasks,
                                                                   char* scratch, uint32_t* counter) {
  __shared__ __align__(16) uint32_t lds[4][RegLds<CW>::kWords];
  uint32_t* mine = lds[(threadIdx.x >> 6) & 3];
  for (;;) {
    const uint32_t k = next_tile(counter);
    if (k >= n) break;
    const BatchTile tl = tiles[order[k]];
    const BatchTask tk = tasks[tl.task];
    const bool mrg = tk.gen == PRAND_MRG32K3A;
    switch (tk.dtype) {
      case PRAND_U32:
        if (mrg) gen_reg<mrg::MrgGen, PRAND_U32, CW>(tl, tk, mine, scratch);
        else gen_reg<lfsr::LfsrGen, PRAND_U32, CW>(tl, tk, mine, scratch);
        break;
      case PRAND_F32:
        if (mrg) gen_reg<mrg::MrgGen, PRAND_F32, CW>(tl, tk, mine, scratch);
        else gen_reg<lfsr::LfsrGen, PRAND_F32, CW>(tl, tk, mine, scratch);
        break;
      default:
        if (mrg) gen_reg<mrg::MrgGen, PRAND_F64, CW>(tl, tk, mine, scratch);
        else gen_reg<lfsr::LfsrGen, PRAND_F64, CW>(tl, tk, mine, scratch);
        break;
    }
    wave_lds_sync();
  }
}

__global__ void __launch_bounds__(256) batch_heavy_kernel(const BatchTile* __restrict__ tiles,
                                                          const uint32_t* __restrict__ order, uint32_t n,
                                                          const BatchTask* __restrict__ tasks, char* scratch,
                                                          uint32_t* counter) {
  __shared__ __align__(16) uint32_t lds[4][gm::LaneRing<gm::kLaneFlushNarrow>::kWaveWords];
  uint32_t* rows = lds[(threadIdx.x >> 6) & 3];
  for (;;) {
    const uint32_t k = next_tile(counter);
    if (k >= n) break;
    const BatchTile tl = tiles[order[k]];
    const BatchTask tk = tasks[tl.task];
    if (tk.gen == PRAND_GQ58X3) {
      switch (tk.dtype) {
        case PRAND_U32: gen_gm_dt<2, PRAND_U32>(tl, tk, scratch, rows); break;
        case PRAND_F32: gen_gm_dt<2, PRAND_F32>(tl, tk, scratch, rows); break;
        default: gen_gm_dt<2, PRAND_F64>(tl, tk, scratch, rows); break;
      }
    } else {
      switch (tk.dtype) {
        case PRAND_U32: gen_gm_dt<1, PRAND_U32>(tl, tk, scratch, rows); break;
        case PRAND_F32: gen_gm_dt<1, PRAND_F32>(tl, tk, scratch, rows); break;
        default: gen_gm_dt<1, PRAND_F64>(tl, tk, scratch, rows); break;
      }
    }
    wave_lds_sync();
  }
}

uint32_t blocks_for(uint32_t ntiles, uint32_t waves) { return (ntiles + waves - 1) / waves; }

// resident workgroups of `waves` wavefronts on the whole chip
template <class K>
uint32_t resident_blocks(K kernel, uint32_t waves, int num_cus) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, (int)(64 * waves), 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return (uint32_t)per_cu * (uint32_t)(num_cus > 0 ? num_cus : 1);
}

}  // namespace

hipError_t launch_batch_reset(uint32_t* counters, hipStream_t st) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, st, counters);
  return hipGetLastError();
}

uint32_t batch_persistent_blocks(int cls, int cw, uint32_t waves, int num_cus) {
  if (cls == kClassHeavy) return resident_blocks(batch_heavy_kernel, waves, num_cus);
  if (cls == kClassLight) return resident_blocks(batch_light_kernel, waves, num_cus);
  return cw == 16 ? resident_blocks(batch_reg_persistent_kernel<16>, waves, num_cus)
                  : resident_blocks(batch_reg_persistent_kernel<32>, waves, num_cus);
}

hipError_t launch_batch_persistent(int cls, int cw, const BatchTile* tiles, const uint32_t* order, uint32_t n,
                                   const BatchTask* tasks, char* scratch, uint32_t* counter, uint32_t waves,
                                   uint32_t blocks, hipStream_t st) {
  if (!n) return hipSuccess;
  // no more workgroups than tiles need
  blocks = std::min<uint32_t>(blocks, blocks_for(n, waves));
  const dim3 grid(blocks), block(64 * waves);
  if (cls == kClassHeavy)
    hipLaunchKernelGGL(batch_heavy_kernel, grid, block, 0, st, tiles, order, n, tasks, scratch, counter);
  else if (cls == kClassLight)
    hipLaunchKernelGGL(batch_light_kernel, grid, block, 0, st, tiles, order, n, tasks, scratch, counter);
  else if (cw == 16)
    hipLaunchKernelGGL(batch_reg_persistent_kernel<16>, grid, block, 0, st, tiles, order, n, tasks, scratch,
                       counter);
  else
    hipLaunchKernelGGL(batch_reg_persistent_kernel<32>, grid, block, 0, st, tiles, order, n, tasks, scratch,
                       counter);
  return hipGetLastError();
}

hipError_t launch_batch_starts(const DeviceTables& T, const BatchTile* tiles, uint32_t ntiles, const BatchTask* tasks,
                               char* scratch, uint32_t waves, hipStream_t st) {
  if (!ntiles) return hipSuccess;
  hipLaunchKernelGGL(batch_starts_kernel, dim3(blocks_for(ntiles, waves)), dim3(64 * waves), 0, st, tiles, ntiles,
                     tasks, scratch, T);
  return hipGetLastError();
}

hipError_t launch_batch_reg(const BatchTile* tiles, uint32_t ntiles, const BatchTask* tasks, const char* scratch,
                            uint32_t waves, hipStream_t st) {
  if (!ntiles) return hipSuccess;
  hipLaunchKernelGGL(batch_reg_kernel, dim3(blocks_for(ntiles, waves)), dim3(64 * waves), 0, st, tiles, ntiles,
                     tasks, scratch);
  return hipGetLastError();
}

hipError_t launch_batch_gm(int shape, const BatchTile* tiles, uint32_t ntiles, const BatchTask* tasks,
                           const char* scratch, uint32_t waves, hipStream_t st) {
  if (!ntiles) return hipSuccess;
  const dim3 grid(blocks_for(ntiles, waves)), block(64 * waves);
  if (shape == 1) hipLaunchKernelGGL(batch_gm_kernel<1>, grid, block, 0, st, tiles, ntiles, tasks, scratch);
  else hipLaunchKernelGGL(batch_gm_kernel<2>, grid, block, 0, st, tiles, ntiles, tasks, scratch);
  return hipGetLastError();
}

hipError_t launch_batch_mt_v1(const BatchTile* mt, uint32_t nmt, const BatchTile* v1, uint32_t nv1,
                              const BatchTask* tasks, char* scratch, uint32_t waves, hipStream_t st) {
  if (!nmt && !nv1) return hipSuccess;
  hipLaunchKernelGGL(batch_mt_v1_kernel, dim3(blocks_for(nmt + nv1, waves)), dim3(64 * waves), 0, st, mt, nmt, v1,
                     nv1, tasks, scratch);
  return hipGetLastError();
}

hipError_t launch_batch_serial(const DeviceTables& T, const BatchTile* tiles, const BatchCounts& n,
                               const BatchTask* tasks, char* scratch, uint32_t waves, hipStream_t st) {
  const BatchTile* reg = tiles;
  const BatchTile* g32 = reg + n.reg;
  const BatchTile* g8 = g32 + n.g32;
  const BatchTile* g3 = g8 + n.g8;
  const BatchTile* mt = g3 + n.g3;
  hipError_t e = launch_batch_starts(T, tiles, n.with_starts(), tasks, scratch, waves, st);
  if (e == hipSuccess && n.mtsec) e = launch_batch_mt_starts(T, mt, n.mt, tasks, scratch, st);
  if (e == hipSuccess) e = launch_batch_mt_v1(mt, n.mt + n.copy, g32, n.g32, tasks, scratch, waves, st);
  if (e == hipSuccess) e = launch_batch_gm(2, g3, n.g3, tasks, scratch, waves, st);
  if (e == hipSuccess) e = launch_batch_gm(1, g8, n.g8, tasks, scratch, waves, st);
  if (e == hipSuccess) e = launch_batch_reg(reg, n.reg, tasks, scratch, waves, st);
  return e;
}

}  // namespace prand
