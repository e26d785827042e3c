// Batched persistent launch: planning, HIP-graph replay and the autotuner.
//
// The planner cuts each task into sections that jump to their first output
// and groups them into per-wavefront tiles (see k_batch.hip); tiles are
// sorted longest first so that the persistent wavefronts finish together.
// The launch (counter reset + persistent kernel) is captured once in a HIP
// graph on a private stream and replayed on the caller's stream.  The
// autotuner times a small grid of (wavefronts per CU, MRG32K3A/LFSR113 lane
// section, GM/GQ group section) on the actual task mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "prand_batch.h"

using namespace prand;

struct prand_batch {
  prand_ctx* ctx = nullptr;
  prand_batch_config cfg{};
  BatchTile* d_tiles = nullptr;
  uint32_t ntiles = 0;
  BatchTask* d_tasks = nullptr;
  uint32_t* d_counter = nullptr;
  uint32_t blocks = 0;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

size_t state_size(int g) {
  switch (g) {
    case PRAND_MT19937: return sizeof(MtState);
    case PRAND_MRG32K3A: return sizeof(MrgState);
    case PRAND_LFSR113: return sizeof(LfsrState);
    default: return sizeof(GmState);
  }
}

// relative wavefront time per output a tile's longest lane sequence costs
double per_output_cost(int gen) {
  switch (gen) {
    case PRAND_MT19937: return 0.35;   // 64 lanes share one stream
    case PRAND_MRG32K3A: return 32;
    case PRAND_LFSR113: return 27;
    case PRAND_GM19:
    case PRAND_GM29: return 11;
    case PRAND_GM31: return 16;
    case PRAND_GM61: return 24;
    case PRAND_GQ58X1: return 20;
    case PRAND_GQ58X3: return 27;
    default: return 25;   // GM55, GQ58.4
  }
}

uint64_t round_up(uint64_t x, uint64_t m) { return (x + m - 1) / m * m; }

void fill_defaults(prand_batch_config& c) {
  if (!c.waves_per_cu) c.waves_per_cu = 16;
  if (!c.reg_section) c.reg_section = 2048;
  if (!c.gm_section) c.gm_section = 4096;
  c.reg_section = (uint32_t)std::max<uint64_t>(32, round_up(c.reg_section, 32));
  c.gm_section = std::max<uint32_t>(32, c.gm_section);
}

void free_batch(prand_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  (void)hipFree(b->d_tiles);
  (void)hipFree(b->d_tasks);
  (void)hipFree(b->d_counter);
  delete b;
}

hipError_t enqueue(prand_batch* b, hipStream_t st) {
  return launch_batch(b->ctx->T, b->d_tiles, b->ntiles, b->d_tasks, b->d_counter, b->blocks, st);
}

std::string signature(prand_ctx* c, const prand_task* tasks, uint32_t ntasks) {
  // task count, then per (generator, dtype): tasks and total outputs (2 digits)
  std::map<int, std::pair<uint64_t, double>> mix;
  for (uint32_t k = 0; k < ntasks; k++) {
    auto& m = mix[tasks[k].gen * 4 + tasks[k].dtype];
    m.first++;
    m.second += (double)tasks[k].n;
  }
  char buf[96];
  std::string s = std::string(c->arch) + "/" + std::to_string(c->num_cus) + "/" + std::to_string(ntasks);
  for (auto& kv : mix) {
    std::snprintf(buf, sizeof buf, "/%d.%d:%llu:%.1e", kv.first / 4, kv.first % 4, (unsigned long long)kv.second.first,
                  kv.second.second);
    s += buf;
  }
  return s;
}

bool cache_lookup(const std::string& key, prand_batch_config* cfg) {
  const char* path = getenv("PRAND_TUNE_CACHE");
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[4096];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    char* tab = std::strchr(line, '\t');
    if (!tab) continue;
    *tab = 0;
    unsigned w, r, g;
    if (key == line && std::sscanf(tab + 1, "%u %u %u", &w, &r, &g) == 3) {
      cfg->waves_per_cu = w;
      cfg->reg_section = r;
      cfg->gm_section = g;
      cfg->use_graph = 1;
      found = true;   // the last entry for a key wins
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(const std::string& key, const prand_batch_config& cfg) {
  const char* path = getenv("PRAND_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s\t%u %u %u\n", key.c_str(), cfg.waves_per_cu, cfg.reg_section, cfg.gm_section);
  std::fclose(f);
}

}  // namespace

namespace prand {

void batch_fill_defaults(prand_batch_config& c) { fill_defaults(c); }

int batch_plan(const prand_task* tasks, uint32_t ntasks, const prand_batch_config& cfg, std::vector<BatchTile>& tiles) {
  std::vector<std::pair<double, BatchTile>> work;
  for (uint32_t k = 0; k < ntasks; k++) {
    const prand_task& t = tasks[k];
    if (t.gen < 0 || t.gen >= PRAND_NUM_GENERATORS || t.dtype < PRAND_U32 || t.dtype > PRAND_F64)
      return PRAND_EINVAL;
    if (!t.state_in || !t.state_out || (t.n && !t.out)) return PRAND_EINVAL;
    if (t.n > (1ull << 40)) return PRAND_ERANGE;
    BatchTile b{};
    b.task = k;
    if (t.n == 0) {
      b.kind = kTileCopy;
      b.len32 = state_size(t.gen) / 4;
      work.push_back({0.0, b});
      continue;
    }
    b.kind = kTileGen;
    const uint64_t n = t.n, es = t.dtype == PRAND_F64 ? 8 : 4;
    const double c = per_output_cost(t.gen);
    if (t.gen == PRAND_MT19937) {
      b.first = 0;
      b.seclen = n;
      b.nsec = 1;
      work.push_back({c * (double)n, b});
      continue;
    }
    if (t.gen == PRAND_MRG32K3A || t.gen == PRAND_LFSR113) {
      uint64_t sec = cfg.reg_section;
      if (n < 64 * sec) sec = std::max<uint64_t>(32, round_up((n + 63) / 64, 32));
      const uint64_t total = (n + sec - 1) / sec;
      b.seclen = sec;
      b.coalesce = ((uintptr_t)t.out % 16 == 0) && ((sec * es) % 16 == 0);
      for (uint64_t f = 0; f < total; f += 64) {
        b.first = f;
        b.nsec = (uint32_t)std::min<uint64_t>(64, total - f);
        work.push_back({c * (double)sec, b});
      }
      continue;
    }
    const bool v1 = t.gen == PRAND_GM19 || t.gen == PRAND_GM29 || t.gen == PRAND_GM31 || t.gen == PRAND_GM61 ||
                    t.gen == PRAND_GQ58X1;
    const uint64_t groups = v1 ? 2 : (t.gen == PRAND_GQ58X3 ? 4 : 8);
    uint64_t sec = cfg.gm_section;
    if (n < groups * sec) sec = std::max<uint64_t>(32, round_up((n + groups - 1) / groups, 32));
    b.seclen = sec;
    if (v1) {
      // both halves of a wavefront run the same number of steps: pair the
      // full sections, give the ragged last section a tile of its own
      const uint64_t full = n / sec, part = n % sec;
      for (uint64_t f = 0; f < full; f += 2) {
        b.first = f;
        b.nsec = (uint32_t)std::min<uint64_t>(2, full - f);
        b.len32 = sec;
        work.push_back({c * (double)sec, b});
      }
      if (part) {
        b.first = full;
        b.nsec = 1;
        b.len32 = part;
        work.push_back({c * (double)part, b});
      }
    } else {
      const uint64_t total = (n + sec - 1) / sec;
      for (uint64_t f = 0; f < total; f += groups) {
        b.first = f;
        b.nsec = (uint32_t)std::min<uint64_t>(groups, total - f);
        work.push_back({c * (double)sec, b});
      }
    }
  }
  if (work.size() > 0xFFFFFFF0ull) return PRAND_ERANGE;
  std::stable_sort(work.begin(), work.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
  tiles.resize(work.size());
  for (size_t i = 0; i < work.size(); i++) tiles[i] = work[i].second;
  return PRAND_OK;
}

}  // namespace prand

extern "C" {

int prand_batch_create(prand_ctx* c, const prand_task* h_tasks, uint32_t ntasks, const prand_batch_config* cfg,
                       prand_batch** out) {
  if (!out) return PRAND_EINVAL;
  *out = nullptr;
  if (!c || (ntasks && !h_tasks)) return PRAND_EINVAL;
  prand_batch_config conf{};
  if (cfg) conf = *cfg;
  fill_defaults(conf);
  std::vector<BatchTile> tiles;
  int rc = batch_plan(h_tasks, ntasks, conf, tiles);
  if (rc) return rc;
  DeviceGuard g(c->device);
  prand_batch* b = new (std::nothrow) prand_batch;
  if (!b) return PRAND_ENOMEM;
  b->ctx = c;
  b->cfg = conf;
  b->ntiles = (uint32_t)tiles.size();
  b->blocks = (uint32_t)std::max<uint64_t>(1, ((uint64_t)c->num_cus * conf.waves_per_cu + 3) / 4);
  hipError_t e = hipMalloc((void**)&b->d_counter, 64);
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_tiles, std::max<size_t>(1, tiles.size()) * sizeof(BatchTile));
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_tasks, std::max<size_t>(1, ntasks) * sizeof(BatchTask));
  if (e == hipSuccess && !tiles.empty())
    e = hipMemcpy(b->d_tiles, tiles.data(), tiles.size() * sizeof(BatchTile), hipMemcpyHostToDevice);
  if (e == hipSuccess && ntasks) e = hipMemcpy(b->d_tasks, h_tasks, ntasks * sizeof(BatchTask), hipMemcpyHostToDevice);
  if (e == hipSuccess && conf.use_graph) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e != hipSuccess) {
    free_batch(b);
    return hipfail(c, e);
  }
  *out = b;
  return PRAND_OK;
}

int prand_batch_tiles(const prand_batch* b, uint32_t* ntiles) {
  if (!b || !ntiles) return PRAND_EINVAL;
  *ntiles = b->ntiles;
  return PRAND_OK;
}

int prand_batch_launch(prand_batch* b, void* stream) {
  if (!b) return PRAND_EINVAL;
  if (b->ntiles == 0) return PRAND_OK;
  DeviceGuard g(b->ctx->device);
  hipStream_t st = (hipStream_t)stream;
  if (!b->cfg.use_graph) {
    hipError_t e = enqueue(b, st);
    return e == hipSuccess ? PRAND_OK : hipfail(b->ctx, e);
  }
  if (!b->exec) {
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t le = enqueue(b, b->cap);
      e = hipStreamEndCapture(b->cap, &b->graph);
      if (e == hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
      return hipfail(b->ctx, e);
    }
  }
  hipError_t e = hipGraphLaunch(b->exec, st);
  return e == hipSuccess ? PRAND_OK : hipfail(b->ctx, e);
}

int prand_batch_destroy(prand_batch* b) {
  if (!b) return PRAND_OK;
  DeviceGuard g(b->ctx->device);
  (void)hipDeviceSynchronize();
  free_batch(b);
  return PRAND_OK;
}

int prand_batch_autotune(prand_ctx* c, const prand_task* h_tasks, uint32_t ntasks, prand_batch_config* best) {
  if (!c || !best || (ntasks && !h_tasks)) return PRAND_EINVAL;
  const std::string key = signature(c, h_tasks, ntasks);
  if (cache_lookup(key, best)) return PRAND_OK;
  DeviceGuard g(c->device);
  // the task buffers may still be in flight on other streams
  hipError_t e = hipDeviceSynchronize();
  hipStream_t st = nullptr;
  hipEvent_t a = nullptr, z = nullptr;
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&z);
  float best_ms = 1e30f;
  prand_batch_config pick{};
  fill_defaults(pick);
  pick.use_graph = 1;
  const uint32_t waves[] = {8, 16, 32};
  const uint32_t regs[] = {512, 2048, 8192};
  const uint32_t gms[] = {1024, 4096, 16384};
  for (uint32_t w : waves)
    for (uint32_t r : regs)
      for (uint32_t gsec : gms) {
        if (e != hipSuccess) break;
        prand_batch_config cand{w, r, gsec, 1};
        prand_batch* b = nullptr;
        int rc = prand_batch_create(c, h_tasks, ntasks, &cand, &b);
        if (rc) {
          if (a) (void)hipEventDestroy(a);
          if (z) (void)hipEventDestroy(z);
          if (st) (void)hipStreamDestroy(st);
          return rc;
        }
        rc = prand_batch_launch(b, st);   // warm-up (and graph capture)
        if (!rc) e = hipEventRecord(a, st);
        for (int i = 0; i < 3 && !rc && e == hipSuccess; i++) rc = prand_batch_launch(b, st);
        if (!rc && e == hipSuccess) e = hipEventRecord(z, st);
        if (!rc && e == hipSuccess) e = hipEventSynchronize(z);
        float ms = 0;
        if (!rc && e == hipSuccess) e = hipEventElapsedTime(&ms, a, z);
        prand_batch_destroy(b);
        if (rc) {
          e = hipErrorUnknown;
          break;
        }
        if (e == hipSuccess && ms < best_ms) {
          best_ms = ms;
          pick = cand;
        }
      }
  if (a) (void)hipEventDestroy(a);
  if (z) (void)hipEventDestroy(z);
  if (st) (void)hipStreamDestroy(st);
  if (e != hipSuccess) return hipfail(c, e);
  *best = pick;
  cache_store(key, pick);
  return PRAND_OK;
}

}  // extern "C"
