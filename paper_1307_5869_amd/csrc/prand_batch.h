// Batched launch: task and tile records shared by the host planner
// (batch.hip) and the batch kernels (k_batch.hip).
#pragma once

#include <vector>

#include "prand_impl.h"

namespace prand {

// one task: the public prand_task, field for field
struct BatchTask {
  int32_t gen;
  int32_t dtype;
  uint64_t n;
  const void* state_in;
  void* state_out;
  void* out;
};
static_assert(sizeof(BatchTask) == sizeof(prand_task), "prand_task layout");

constexpr uint32_t kTileGen = 0;    // generate sections first .. first + nsec - 1
constexpr uint32_t kTileCopy = 1;   // n = 0: copy state_in to state_out
// section `first` of a long MT19937 task (kMtSection outputs each: whole
// 624-word blocks), started from the state the section-start kernel leaves
// in the scratch
constexpr uint32_t kTileMtSection = 2;
constexpr uint64_t kMtSection = 624ull << kMtBlkFirst;

// the work of one wavefront
struct BatchTile {
  uint32_t task;
  uint32_t kind;
  uint64_t first;      // first section of the tile
  uint64_t seclen;     // outputs per section (the task's last section may be shorter)
  uint32_t nsec;       // live sections in the tile
  uint32_t coalesce;   // MRG32K3A/LFSR113: every section start 16-byte aligned
  uint64_t len32;      // v = 1 GM/GQ tiles: the common length of the live
                       // sections; copy tiles: 32-bit words of the state
  uint64_t starts;     // byte offset of the tile's section start states in
                       // the batch scratch (MRG32K3A/LFSR113 and GM/GQ tiles)
};

// tiles are stored family by family: [reg | g32 | g8 | g3 | mt | copy]
// (MRG32K3A/LFSR113; GM/GQ with v = 1, with v = 4, GQ58.3; MT19937; n = 0)
struct BatchCounts {
  uint32_t reg = 0, g32 = 0, g8 = 0, g3 = 0, mt = 0, copy = 0;
  uint32_t mtsec = 0;   // MT19937 section tiles among the mt ones
  uint32_t with_starts() const { return reg + g32 + g8 + g3; }
  uint32_t total() const { return with_starts() + mt + copy; }
};
constexpr int kBatchFamilies = 6;

struct BatchPlan {
  std::vector<BatchTile> tiles;
  BatchCounts n;
  uint64_t scratch_bytes = 0;
  // tile indices of the register classes of the persistent launch, longest
  // (estimated wavefront time) first: light = v = 1 GM/GQ, MT19937, copies;
  // reg = MRG32K3A/LFSR113; heavy = v = 4 GM/GQ, GQ58.3
  std::vector<uint32_t> order_light, order_reg, order_heavy;
  // estimated wavefront time of each class's tiles, summed (the planner's
  // relative cost units), indexed by kClass*
  double cost[3] = {0, 0, 0};
};

// zero fields of a configuration replaced by the defaults
void batch_fill_defaults(prand_batch_config& c);
// cut tasks into tiles, family by family, each family longest first
// (PRAND_OK or an error code); MT19937 tasks longer than mt_section_min
// outputs are cut into kMtSection-output sections
int batch_plan(const prand_task* tasks, uint32_t ntasks, const prand_batch_config& cfg, BatchPlan& plan,
               uint64_t mt_section_min);
// MT19937 tasks of a batched launch above this many outputs (about 16 ms of
// one wavefront) run as sections; below it the jumps cost more than the
// wavefront's run, which the batch's other work covers
constexpr uint64_t kMtBatchSectionMin = 1ull << 24;

// the kernels of a batch, `waves` wavefronts (tiles) per workgroup
hipError_t launch_batch_starts(const DeviceTables& T, const BatchTile* tiles, uint32_t ntiles, const BatchTask* tasks,
                               char* scratch, uint32_t waves, hipStream_t st);
hipError_t launch_batch_reg(const BatchTile* tiles, uint32_t ntiles, const BatchTask* tasks, const char* scratch,
                            uint32_t waves, hipStream_t st);
// lane-section GM/GQ shapes: 1 = v = 4 ensembles, 2 = GQ58.3
hipError_t launch_batch_gm(int shape, const BatchTile* tiles, uint32_t ntiles, const BatchTask* tasks,
                           const char* scratch, uint32_t waves, hipStream_t st);
// MT19937 tiles (and n = 0 copies) followed by the v = 1 GM/GQ tiles, in one
// launch (after the section starts, which the v = 1 and MT19937 section
// tiles read)
hipError_t launch_batch_mt_v1(const BatchTile* mt, uint32_t nmt, const BatchTile* v1, uint32_t nv1,
                              const BatchTask* tasks, char* scratch, uint32_t waves, hipStream_t st);
// start states of the MT19937 section tiles among tiles[0 .. ntiles): the
// task state moved first * kMtSection outputs on (one wavefront each)
hipError_t launch_batch_mt_starts(const DeviceTables& T, const BatchTile* tiles, uint32_t ntiles,
                                  const BatchTask* tasks, char* scratch, hipStream_t st);
// persistent launch: one tile counter per class, cleared by a small kernel
// (no memset node in a captured graph)
constexpr int kClassLight = 0, kClassReg = 1, kClassHeavy = 2;
constexpr int kBatchCounters = 3;
hipError_t launch_batch_reset(uint32_t* counters, hipStream_t st);
// workgroups of `waves` wavefronts of a class's persistent kernel (reg: LDS
// chunk width cw = 16 or 32) resident on the chip at once
uint32_t batch_persistent_blocks(int cls, int cw, uint32_t waves, int num_cus);
hipError_t launch_batch_persistent(int cls, int cw, const BatchTile* tiles, const uint32_t* order, uint32_t n,
                                   const BatchTask* tasks, char* scratch, uint32_t* counter, uint32_t waves,
                                   uint32_t blocks, hipStream_t st);
// all of them on one stream: section starts, MT19937 + v = 1, the other GM/GQ, MRG32K3A/LFSR113
hipError_t launch_batch_serial(const DeviceTables& T, const BatchTile* tiles, const BatchCounts& n,
                               const BatchTask* tasks, char* scratch, uint32_t waves, hipStream_t st);

}  // namespace prand
