// Batched persistent launch: task and tile records shared by the host
// planner (batch.hip) and the persistent kernel (k_batch.hip).
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
};

// zero fields of a configuration replaced by the defaults
void batch_fill_defaults(prand_batch_config& c);
// cut tasks into tiles, longest first (PRAND_OK or an error code)
int batch_plan(const prand_task* tasks, uint32_t ntasks, const prand_batch_config& cfg, std::vector<BatchTile>& tiles);

hipError_t launch_batch(const DeviceTables& T, const BatchTile* tiles, uint32_t ntiles, const BatchTask* tasks,
                        uint32_t* counter, uint32_t blocks, hipStream_t st);

}  // namespace prand
