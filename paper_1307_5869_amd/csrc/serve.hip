// Serving loop: continuous batching of generate requests over one device.
//
// One worker thread owns the device work.  Requests are served in two lanes
// that run concurrently on their own HIP streams: MT19937 (one wavefront per
// chunk, so its chunks are long) and every other generator.  Each turn of
// the worker's loop it
//  1. takes newly submitted requests into a FIFO of waiting requests and
//     applies the releases clients have made;
//  2. reports the requests whose last chunk a finished launch held as
//     complete, and marks the requests of a finished initialisation ready;
//  3. per lane, when no initialisation is in flight, admits waiting requests
//     while their output and two state slots fit in the HBM arena reserved at
//     creation (a later request may pass an earlier one that does not fit,
//     unless the earlier one has waited too long), and initialises their
//     streams by block splitting: one jump launch per (generator, variant)
//     group into a staging area, then a scatter into each request's first
//     state slot;
//  4. per lane, with fewer than two launches in flight, enqueues one loop
//     iteration: a batched launch (the batch kernels, in order on the lane's
//     stream) holding the next chunk of every ready request of the lane.  Chunks are an equal share of the
//     iteration's output budget (never below the minimum chunk; MT19937
//     chunks are capped); a request's state ping-pongs between its two slots,
//     so consecutive chunks continue the stream exactly.
// Completion is observed by polling events, so one lane never waits for the
// other.  Outputs and final states stay in the arena until released.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "prand_batch.h"

using namespace prand;

namespace {

constexpr uint32_t kInitMax = 4096;          // requests per initialisation batch
constexpr uint32_t kInitItems = 16384;       // state slots filled per initialisation batch
constexpr size_t kStateSlot = 2560;          // bytes per staged state (>= every state blob)
constexpr uint64_t kAlign = 256;
constexpr double kStarveS = 0.05;            // a waiting request older than this blocks bypassing

size_t state_size(int g) {
  switch (g) {
    case PRAND_MT19937: return sizeof(MtState);
    case PRAND_MRG32K3A: return sizeof(MrgState);
    case PRAND_LFSR113: return sizeof(LfsrState);
    default: return sizeof(GmState);
  }
}
uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// first-fit allocator over [0, size) with coalescing of free neighbours
class Arena {
 public:
  void reset(uint64_t size) {
    free_.clear();
    if (size) free_[0] = size;
    size_ = size;
    used_ = peak_ = 0;
  }
  bool alloc(uint64_t bytes, uint64_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const uint64_t rest = it->second - bytes;
      const uint64_t start = it->first + bytes;
      free_.erase(it);
      if (rest) free_[start] = rest;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return true;
    }
    return false;
  }
  void release(uint64_t off, uint64_t bytes) {
    used_ -= bytes;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }
  uint64_t size() const { return size_; }
  uint64_t used() const { return used_; }
  uint64_t peak() const { return peak_; }

 private:
  std::map<uint64_t, uint64_t> free_;
  uint64_t size_ = 0, used_ = 0, peak_ = 0;
};

// A contiguous run of a request's outputs, generated from its own state: a
// request is one section, or (long MT19937 requests) up to kMaxSections that
// start from jumped states and run in parallel.
struct Section {
  uint64_t start = 0, len = 0;
  uint64_t issued = 0;           // outputs of the section enqueued
  char* st[2] = {nullptr, nullptr};
  int cur = 0;                   // slot holding the state after the enqueued chunks
};

struct Req {
  uint64_t ticket = 0;
  prand_request r{};
  double t_submit = 0, t_admit = 0, t_done = 0;
  uint64_t off = 0, bytes = 0;   // arena block: output, then the sections' state slots
  char* out = nullptr;
  std::vector<Section> secs;
  uint64_t seclen = 0;           // outputs per section (all but the last)
  uint64_t issued = 0;           // outputs enqueued over all sections
  bool ready = false;            // streams initialised
  bool complete = false;         // last chunk finished
};

constexpr uint32_t kMaxSections = 256;
// shortest MT19937 section: 624 * 2^kMinSectionLog2 outputs, about 1.3 ms
// on the one wavefront that generates a section
constexpr int kMinSectionLog2 = 10;
static_assert(kMinSectionLog2 >= kMtBlkFirst, "sections are whole-block-table units");

struct ScatterItem {
  const uint32_t* src;
  uint32_t* dst;
  uint64_t words;
};

__global__ void scatter_states_kernel(const ScatterItem* __restrict__ items, uint32_t count) {
  const uint32_t i = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (i >= count) return;
  const ScatterItem it = items[i];
  for (uint64_t w = threadIdx.x & 63; w < it.words; w += 64) it.dst[w] = it.src[w];
}

struct InitBatch {
  uint64_t* h_ids = nullptr;     // pinned
  uint64_t* d_ids = nullptr;
  uint64_t* h_dist = nullptr;    // pinned: section start distances
  uint64_t* d_dist = nullptr;
  char* d_staging = nullptr;
  ScatterItem* h_items = nullptr;  // pinned
  ScatterItem* d_items = nullptr;
  hipEvent_t ev = nullptr;
  std::vector<Req*> reqs;
  bool in_flight = false;
};

struct IterSlot {
  prand_task* h_tasks = nullptr;   // pinned
  BatchTask* d_tasks = nullptr;
  BatchTile* h_tiles = nullptr;    // pinned
  BatchTile* d_tiles = nullptr;
  uint32_t task_cap = 0, tile_cap = 0;
  char* d_scratch = nullptr;     // section start states of the iteration's tiles
  uint64_t scratch_cap = 0;
  hipEvent_t start = nullptr, end = nullptr;
  std::vector<Req*> finishing;
  bool in_flight = false;
  uint64_t seq = 0;
};

// MT19937 requests, and all the others
constexpr int kLanes = 2;
int lane_of(int gen) { return gen == PRAND_MT19937 ? 0 : 1; }

struct Lane {
  hipStream_t init_st = nullptr, gen_st = nullptr;
  InitBatch init;
  IterSlot slot[2];
  std::vector<Req*> active;      // admitted, not complete
  uint64_t iter_seq = 0;
};

}  // namespace

struct prand_server {
  prand_ctx* ctx = nullptr;
  prand_server_config cfg{};
  prand_batch_config bcfg{};
  std::chrono::steady_clock::time_point t0;

  std::thread worker;
  std::mutex mu;                       // guards everything below up to the worker-only part
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  int error = 0;                       // sticky PRAND_E* once the worker failed
  uint64_t next_ticket = 1;
  std::deque<Req*> inbox;
  std::deque<prand_completion> done;
  std::unordered_map<uint64_t, Req*> finished;   // completed, not yet released
  std::vector<uint64_t> release_q;
  Arena arena;
  prand_server_stats st{};

  // worker only
  char* d_arena = nullptr;
  std::deque<Req*> waiting;
  Lane lane[kLanes];
  BatchPlan plan;
  std::vector<prand_task> tasks;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

void fill_config(prand_server_config& c) {
  if (!c.hbm_budget) c.hbm_budget = 16ull << 30;
  if (!c.iter_numbers) c.iter_numbers = 1ull << 28;
  if (!c.min_chunk) c.min_chunk = 1ull << 16;
  if (!c.mt_chunk) c.mt_chunk = 1ull << 20;
  if (!c.mt_section) c.mt_section = 1ull << 20;
  if (!c.max_active) c.max_active = 8192;
  if (!c.max_queue) c.max_queue = 1u << 20;
}

// Sections of a request: MT19937 requests longer than mt_section are cut into
// at most kMaxSections of 624 * 2^k outputs (k >= kMinSectionLog2), so that every section
// starts on a twist-block boundary of the stream (block-splitting states sit
// on one) and its start distance has few set bits.  A jump yields the
// canonical state, which differs from the sequentially reached one only in
// bits the next twist overwrites; since every section starts with a twist,
// outputs and the last section's final state equal sequential generation.
uint64_t section_len(const prand_request& r, const prand_server_config& cfg) {
  if (r.gen != PRAND_MT19937 || r.n <= cfg.mt_section) return r.n;
  uint64_t len = 624ull << kMinSectionLog2;
  while ((r.n + len - 1) / len > kMaxSections) len <<= 1;
  return len;
}
uint32_t section_count(const prand_request& r, const prand_server_config& cfg) {
  const uint64_t len = section_len(r, cfg);
  return (uint32_t)((r.n + len - 1) / len);
}

// arena block of a request: output, then the sections' first state slots
// (contiguous, one state apart), then their second slots
uint64_t request_bytes(const prand_request& r, const prand_server_config& cfg) {
  const uint64_t es = r.dtype == PRAND_F64 ? 8 : 4;
  const uint64_t slots = align_up((uint64_t)section_count(r, cfg) * state_size(r.gen));
  return align_up(r.n * es) + 2 * slots;
}

void layout_request(Req* r, char* base, const prand_server_config& cfg) {
  const uint64_t es = r->r.dtype == PRAND_F64 ? 8 : 4;
  const uint32_t ns = section_count(r->r, cfg);
  const size_t sb = state_size(r->r.gen);
  const uint64_t slots = align_up((uint64_t)ns * sb);
  r->out = base;
  r->seclen = section_len(r->r, cfg);
  r->secs.assign(ns, Section{});
  char* a = base + align_up(r->r.n * es);
  for (uint32_t j = 0; j < ns; j++) {
    Section& q = r->secs[j];
    q.start = (uint64_t)j * r->seclen;
    q.len = std::min<uint64_t>(r->seclen, r->r.n - q.start);
    q.st[0] = a + (size_t)j * sb;
    q.st[1] = a + slots + (size_t)j * sb;
  }
}

hipError_t grow_slot(prand_server* s, IterSlot& sl, uint32_t ntasks, uint32_t ntiles, uint64_t scratch) {
  if (ntasks <= sl.task_cap && ntiles <= sl.tile_cap && scratch <= sl.scratch_cap) return hipSuccess;
  // the slot is idle (its last launch has been waited for)
  hipError_t e = hipSuccess;
  if (ntasks > sl.task_cap) {
    const uint32_t cap = std::max<uint32_t>(ntasks, sl.task_cap * 2);
    (void)hipHostFree(sl.h_tasks);
    (void)hipFree(sl.d_tasks);
    sl.h_tasks = nullptr;
    sl.d_tasks = nullptr;
    sl.task_cap = 0;
    e = hipHostMalloc((void**)&sl.h_tasks, cap * sizeof(prand_task), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&sl.d_tasks, cap * sizeof(BatchTask));
    if (e == hipSuccess) sl.task_cap = cap;
  }
  if (e == hipSuccess && ntiles > sl.tile_cap) {
    const uint32_t cap = std::max<uint32_t>(ntiles, sl.tile_cap * 2);
    (void)hipHostFree(sl.h_tiles);
    (void)hipFree(sl.d_tiles);
    sl.h_tiles = nullptr;
    sl.d_tiles = nullptr;
    sl.tile_cap = 0;
    e = hipHostMalloc((void**)&sl.h_tiles, cap * sizeof(BatchTile), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&sl.d_tiles, cap * sizeof(BatchTile));
    if (e == hipSuccess) sl.tile_cap = cap;
  }
  if (e == hipSuccess && scratch > sl.scratch_cap) {
    const uint64_t cap = std::max<uint64_t>(scratch, sl.scratch_cap * 2);
    (void)hipFree(sl.d_scratch);
    sl.d_scratch = nullptr;
    sl.scratch_cap = 0;
    e = hipMalloc((void**)&sl.d_scratch, cap);
    if (e == hipSuccess) sl.scratch_cap = cap;
  }
  (void)s;
  return e;
}

size_t active_total(const prand_server* s) {
  size_t n = 0;
  for (const Lane& l : s->lane) n += l.active.size();
  return n;
}

// Admit waiting requests of lane li (memory, activity and batch limits) and
// enqueue their stream initialisation.  Worker thread; takes s->mu for the
// arena and the active lists.
int admit_and_init(prand_server* s, int li) {
  Lane& L = s->lane[li];
  InitBatch& ib = L.init;
  ib.reqs.clear();
  if (s->waiting.empty()) return PRAND_OK;
  const double t = s->now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    const size_t act = active_total(s);
    size_t limit = s->cfg.max_active > act ? s->cfg.max_active - act : 0;
    limit = std::min<size_t>(limit, kInitMax);
    uint32_t items = 0;
    for (auto it = s->waiting.begin(); it != s->waiting.end() && ib.reqs.size() < limit;) {
      Req* r = *it;
      if (lane_of(r->r.gen) != li) {
        ++it;
        continue;
      }
      const uint32_t ns = section_count(r->r, s->cfg);
      if (items + ns > kInitItems) break;
      uint64_t off;
      if (s->arena.alloc(r->bytes, &off)) {
        r->off = off;
        layout_request(r, s->d_arena + off, s->cfg);
        items += ns;
        r->t_admit = t;
        ib.reqs.push_back(r);
        it = s->waiting.erase(it);
        s->st.admitted++;
      } else {
        if (t - r->t_submit > kStarveS) break;   // keep the memory for the oldest
        ++it;
      }
    }
    for (Req* r : ib.reqs) L.active.push_back(r);
    s->st.hbm_used = s->arena.used();
    s->st.hbm_peak = s->arena.peak();
  }
  if (ib.reqs.empty()) return PRAND_OK;
  // group by (generator, variant): each group's jump writes its states packed
  // at the group's state size from the staging slot of its first request
  std::stable_sort(ib.reqs.begin(), ib.reqs.end(), [](const Req* a, const Req* b) {
    return a->r.gen != b->r.gen ? a->r.gen < b->r.gen : a->r.variant < b->r.variant;
  });
  const uint32_t n = (uint32_t)ib.reqs.size();
  std::vector<uint32_t> group_start;
  uint32_t items = 0, dists = 0;
  for (uint32_t i = 0; i < n; i++) {
    const Req* r = ib.reqs[i];
    if (i == 0 || r->r.gen != ib.reqs[i - 1]->r.gen || r->r.variant != ib.reqs[i - 1]->r.variant)
      group_start.push_back(i);
    const uint32_t a = group_start.back();
    const size_t sb = state_size(r->r.gen);
    ib.h_ids[i] = r->r.stream_id;
    // every section's first slot starts as the stream's state
    for (const Section& q : r->secs) {
      ib.h_items[items].src = (const uint32_t*)(ib.d_staging + (size_t)a * kStateSlot + (size_t)(i - a) * sb);
      ib.h_items[items].dst = (uint32_t*)q.st[0];
      ib.h_items[items].words = sb / 4;
      items++;
    }
    // section starts in whole sections of 624 2^kMtBlkFirst outputs (every
    // section length is a multiple of one)
    if (r->secs.size() > 1)
      for (const Section& q : r->secs) ib.h_dist[dists++] = q.start / kMtSection;
  }
  group_start.push_back(n);
  hipError_t e = hipMemcpyAsync(ib.d_ids, ib.h_ids, n * sizeof(uint64_t), hipMemcpyHostToDevice, L.init_st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ib.d_items, ib.h_items, items * sizeof(ScatterItem), hipMemcpyHostToDevice, L.init_st);
  if (e == hipSuccess && dists)
    e = hipMemcpyAsync(ib.d_dist, ib.h_dist, dists * sizeof(uint64_t), hipMemcpyHostToDevice, L.init_st);
  if (e != hipSuccess) return hipfail(s->ctx, e);
  for (size_t k = 0; k + 1 < group_start.size(); k++) {
    const uint32_t a = group_start[k], b = group_start[k + 1];
    int rc = prand_init_streams_dev(s->ctx, ib.reqs[a]->r.gen, ib.reqs[a]->r.variant, nullptr, ib.d_ids + a, b - a,
                                    ib.d_staging + (size_t)a * kStateSlot, L.init_st);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(scatter_states_kernel, dim3((items + 3) / 4), dim3(256), 0, L.init_st, ib.d_items, items);
  e = hipGetLastError();
  // sectioned requests: move each section's copy to its start, in place
  uint32_t d0 = 0;
  for (uint32_t i = 0; i < n && e == hipSuccess; i++) {
    const Req* r = ib.reqs[i];
    if (r->secs.size() <= 1) continue;
    JumpSpec js;
    js.dist = ib.d_dist + d0;
    js.nlimbs = 1;
    js.per_stream = 1;
    js.mt_blocks = 1;
    e = launch_mt_jump(s->ctx->T, (MtState*)r->secs[0].st[0], (uint32_t)r->secs.size(), js, nullptr, L.init_st);
    d0 += (uint32_t)r->secs.size();
  }
  if (e == hipSuccess) e = hipEventRecord(ib.ev, L.init_st);
  if (e != hipSuccess) return hipfail(s->ctx, e);
  ib.in_flight = true;
  return PRAND_OK;
}

// one loop iteration of lane L into its slot sl; *launched is false when no
// request of the lane has work
int enqueue_iteration(prand_server* s, Lane& L, IterSlot& sl, bool* launched) {
  *launched = false;
  uint64_t m = 0;
  for (Req* r : L.active)
    if (r->ready)
      for (const Section& q : r->secs) m += q.issued < q.len;
  if (m == 0) return PRAND_OK;
  const uint64_t share = std::max<uint64_t>(s->cfg.min_chunk, s->cfg.iter_numbers / m);
  s->tasks.clear();
  sl.finishing.clear();
  for (Req* r : L.active) {
    if (!r->ready || r->issued >= r->r.n) continue;
    const uint64_t es = r->r.dtype == PRAND_F64 ? 8 : 4;
    for (Section& q : r->secs) {
      if (q.issued >= q.len) continue;
      uint64_t chunk = std::min<uint64_t>(q.len - q.issued, share);
      if (r->r.gen == PRAND_MT19937) chunk = std::min<uint64_t>(chunk, s->cfg.mt_chunk);
      prand_task t;
      t.gen = r->r.gen;
      t.dtype = r->r.dtype;
      t.n = chunk;
      t.state_in = q.st[q.cur];
      t.state_out = q.st[q.cur ^ 1];
      t.out = r->out + (q.start + q.issued) * es;
      s->tasks.push_back(t);
      q.cur ^= 1;
      q.issued += chunk;
      r->issued += chunk;
    }
    if (r->issued == r->r.n) sl.finishing.push_back(r);
  }
  BatchPlan& plan = s->plan;
  // MT19937 requests are sectioned at admission; their chunks stay whole
  int rc = batch_plan(s->tasks.data(), (uint32_t)s->tasks.size(), s->bcfg, plan, UINT64_MAX);
  if (rc) return rc;
  hipError_t e = grow_slot(s, sl, (uint32_t)s->tasks.size(), (uint32_t)plan.tiles.size(), plan.scratch_bytes);
  if (e != hipSuccess) return hipfail(s->ctx, e);
  std::memcpy(sl.h_tasks, s->tasks.data(), s->tasks.size() * sizeof(prand_task));
  std::memcpy(sl.h_tiles, plan.tiles.data(), plan.tiles.size() * sizeof(BatchTile));
  e = hipMemcpyAsync(sl.d_tasks, sl.h_tasks, s->tasks.size() * sizeof(BatchTask), hipMemcpyHostToDevice, L.gen_st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(sl.d_tiles, sl.h_tiles, plan.tiles.size() * sizeof(BatchTile), hipMemcpyHostToDevice, L.gen_st);
  if (e == hipSuccess) e = hipEventRecord(sl.start, L.gen_st);
  if (e == hipSuccess)
    e = launch_batch_serial(s->ctx->T, sl.d_tiles, plan.n, sl.d_tasks, sl.d_scratch, s->bcfg.waves_per_block,
                            L.gen_st);
  if (e == hipSuccess) e = hipEventRecord(sl.end, L.gen_st);
  if (e != hipSuccess) return hipfail(s->ctx, e);
  sl.in_flight = true;
  sl.seq = ++L.iter_seq;
  *launched = true;
  return PRAND_OK;
}

// slot sl of lane L has finished: report the requests it completed
int finish_slot(prand_server* s, Lane& L, IterSlot& sl) {
  const double t = s->now();
  float ms = 0;
  (void)hipEventElapsedTime(&ms, sl.start, sl.end);
  sl.in_flight = false;
  std::lock_guard<std::mutex> lk(s->mu);
  s->st.iterations++;
  s->st.gpu_busy_s += ms * 1e-3;
  for (Req* r : sl.finishing) {
    r->t_done = t;
    r->complete = true;
    prand_completion c;
    c.ticket = r->ticket;
    c.tag = r->r.tag;
    c.n = r->r.n;
    c.gen = r->r.gen;
    c.dtype = r->r.dtype;
    c.out = r->out;
    c.state = r->secs.back().st[r->secs.back().cur];
    c.t_submit = r->t_submit;
    c.t_admit = r->t_admit;
    c.t_done = t;
    s->done.push_back(c);
    s->finished[r->ticket] = r;
    s->st.completed++;
    s->st.numbers += r->r.n;
  }
  if (!sl.finishing.empty()) {
    L.active.erase(std::remove_if(L.active.begin(), L.active.end(), [](const Req* r) { return r->complete; }),
                   L.active.end());
    s->cv_done.notify_all();
  }
  sl.finishing.clear();
  return PRAND_OK;
}

// 1 when the event has completed, 0 when not yet, an error code otherwise
int event_done(prand_server* s, hipEvent_t ev) {
  const hipError_t e = hipEventQuery(ev);
  if (e == hipSuccess) return 1;
  if (e == hipErrorNotReady) return 0;
  return hipfail(s->ctx, e);
}

// one turn of the worker: returns PRAND_OK and sets *progress when anything
// moved
int worker_turn(prand_server* s, bool* progress) {
  *progress = false;
  for (Lane& L : s->lane) {
    // finished launches, oldest first
    for (;;) {
      IterSlot* oldest = nullptr;
      for (IterSlot& sl : L.slot)
        if (sl.in_flight && (!oldest || sl.seq < oldest->seq)) oldest = &sl;
      if (!oldest) break;
      const int d = event_done(s, oldest->end);
      if (d < 0) return d;
      if (!d) break;
      int rc = finish_slot(s, L, *oldest);
      if (rc) return rc;
      *progress = true;
    }
    // finished initialisation: those requests may generate
    if (L.init.in_flight) {
      const int d = event_done(s, L.init.ev);
      if (d < 0) return d;
      if (d) {
        for (Req* r : L.init.reqs) r->ready = true;
        L.init.in_flight = false;
        L.init.reqs.clear();
        *progress = true;
      }
    }
  }
  for (int li = 0; li < kLanes; li++) {
    Lane& L = s->lane[li];
    if (!L.init.in_flight && !s->waiting.empty()) {
      int rc = admit_and_init(s, li);
      if (rc) return rc;
      if (L.init.in_flight) *progress = true;
    }
    IterSlot* free_slot = !L.slot[0].in_flight ? &L.slot[0] : (!L.slot[1].in_flight ? &L.slot[1] : nullptr);
    if (free_slot) {
      bool launched = false;
      int rc = enqueue_iteration(s, L, *free_slot, &launched);
      if (rc) return rc;
      if (launched) *progress = true;
    }
  }
  return PRAND_OK;
}

void worker_main(prand_server* s) {
  DeviceGuard g(s->ctx->device);
  int rc = PRAND_OK;
  for (;;) {
    bool device_busy = false;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      for (uint64_t t : s->release_q) {
        auto it = s->finished.find(t);
        if (it == s->finished.end()) continue;
        s->arena.release(it->second->off, it->second->bytes);
        delete it->second;
        s->finished.erase(it);
        s->st.released++;
      }
      s->release_q.clear();
      s->st.hbm_used = s->arena.used();
      while (!s->inbox.empty()) {
        s->waiting.push_back(s->inbox.front());
        s->inbox.pop_front();
      }
      if (s->stop) {
        for (Req* r : s->waiting) delete r;   // never admitted
        s->waiting.clear();
      }
      s->st.waiting = (uint32_t)s->waiting.size();
      s->st.active = (uint32_t)active_total(s);
      for (const Lane& L : s->lane)
        device_busy |= L.init.in_flight || L.slot[0].in_flight || L.slot[1].in_flight || !L.active.empty();
      if (!device_busy && s->waiting.empty()) {
        if (s->stop) break;
        s->cv_work.wait_for(lk, std::chrono::milliseconds(20));
        continue;
      }
    }
    bool progress = false;
    rc = worker_turn(s, &progress);
    if (rc) break;
    if (!progress) {
      if (device_busy) {
        // launches in flight: poll again shortly
        std::this_thread::sleep_for(std::chrono::microseconds(20));
      } else {
        // requests wait for memory and nothing runs: wait for a release
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->release_q.empty() && s->inbox.empty() && !s->stop)
          s->cv_work.wait_for(lk, std::chrono::milliseconds(2));
      }
    }
  }
  if (rc) {
    for (Lane& L : s->lane) {
      (void)hipStreamSynchronize(L.gen_st);
      (void)hipStreamSynchronize(L.init_st);
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->error = rc;
    s->cv_done.notify_all();
  }
}

void free_server(prand_server* s) {
  if (!s) return;
  DeviceGuard g(s->ctx->device);
  for (Lane& L : s->lane) {
    if (L.gen_st) (void)hipStreamSynchronize(L.gen_st);
    if (L.init_st) (void)hipStreamSynchronize(L.init_st);
  }
  for (Lane& L : s->lane) {
    for (IterSlot& sl : L.slot) {
      (void)hipHostFree(sl.h_tasks);
      (void)hipHostFree(sl.h_tiles);
      (void)hipFree(sl.d_tasks);
      (void)hipFree(sl.d_tiles);
      (void)hipFree(sl.d_scratch);
      if (sl.start) (void)hipEventDestroy(sl.start);
      if (sl.end) (void)hipEventDestroy(sl.end);
    }
    InitBatch& ib = L.init;
    (void)hipHostFree(ib.h_ids);
    (void)hipHostFree(ib.h_items);
    (void)hipHostFree(ib.h_dist);
    (void)hipFree(ib.d_dist);
    (void)hipFree(ib.d_ids);
    (void)hipFree(ib.d_items);
    (void)hipFree(ib.d_staging);
    if (ib.ev) (void)hipEventDestroy(ib.ev);
    if (L.gen_st) (void)hipStreamDestroy(L.gen_st);
    if (L.init_st) (void)hipStreamDestroy(L.init_st);
    for (Req* r : L.active) delete r;
  }
  (void)hipFree(s->d_arena);
  for (Req* r : s->waiting) delete r;
  for (Req* r : s->inbox) delete r;
  for (auto& kv : s->finished) delete kv.second;
  delete s;
}

}  // namespace

extern "C" {

int prand_server_create(prand_ctx* c, const prand_server_config* cfg, prand_server** out) {
  if (!out) return PRAND_EINVAL;
  *out = nullptr;
  if (!c) return PRAND_EINVAL;
  prand_server* s = new (std::nothrow) prand_server;
  if (!s) return PRAND_ENOMEM;
  s->ctx = c;
  if (cfg) s->cfg = *cfg;
  fill_config(s->cfg);
  s->bcfg.waves_per_block = s->cfg.waves_per_block;
  s->bcfg.reg_section = s->cfg.reg_section;
  s->bcfg.gm_section = s->cfg.gm_section;
  batch_fill_defaults(s->bcfg);
  s->t0 = std::chrono::steady_clock::now();
  DeviceGuard g(c->device);
  hipError_t e = hipMalloc((void**)&s->d_arena, s->cfg.hbm_budget);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    delete s;
    return PRAND_ENOMEM;
  }
  s->arena.reset(s->cfg.hbm_budget);
  s->st.hbm_budget = s->cfg.hbm_budget;
  for (Lane& L : s->lane) {
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&L.gen_st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&L.init_st, hipStreamNonBlocking);
    InitBatch& ib = L.init;
    if (e == hipSuccess) e = hipHostMalloc((void**)&ib.h_ids, kInitMax * sizeof(uint64_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&ib.h_items, kInitItems * sizeof(ScatterItem), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&ib.h_dist, kInitItems * sizeof(uint64_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&ib.d_ids, kInitMax * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMalloc((void**)&ib.d_items, kInitItems * sizeof(ScatterItem));
    if (e == hipSuccess) e = hipMalloc((void**)&ib.d_dist, kInitItems * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMalloc((void**)&ib.d_staging, kInitMax * kStateSlot);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ib.ev, hipEventDisableTiming);
    for (IterSlot& sl : L.slot) {
      if (e == hipSuccess) e = hipEventCreate(&sl.start);
      if (e == hipSuccess) e = hipEventCreate(&sl.end);
      if (e == hipSuccess) e = grow_slot(s, sl, 1024, 16384, 16384 * 1536);
    }
  }
  if (e != hipSuccess) {
    free_server(s);
    return hipfail(c, e);
  }
  // MT19937 stream initialisation needs its polynomial tables: build them
  // now rather than inside the first MT19937 request's latency
  int rc = ensure_mt_tables(c);
  if (rc) {
    free_server(s);
    return rc;
  }
  try {
    s->worker = std::thread(worker_main, s);
  } catch (...) {
    free_server(s);
    return PRAND_ENOMEM;
  }
  *out = s;
  return PRAND_OK;
}

int prand_server_submit(prand_server* s, const prand_request* req, uint64_t* ticket) {
  if (!s || !req || !ticket) return PRAND_EINVAL;
  const prand_request& r = *req;
  if (r.gen < 0 || r.gen >= PRAND_NUM_GENERATORS || r.dtype < PRAND_U32 || r.dtype > PRAND_F64) return PRAND_EINVAL;
  if (r.n == 0) return PRAND_EINVAL;
  const int be = prand_block_log2(r.gen, r.variant);
  if (be < 0) return be;
  if (r.n > (1ull << 40) || request_bytes(r, s->cfg) > s->cfg.hbm_budget) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->st.rejected++;
    return PRAND_ERANGE;
  }
  Req* q = new (std::nothrow) Req;
  if (!q) return PRAND_ENOMEM;
  q->r = r;
  q->bytes = request_bytes(r, s->cfg);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->error) {
      delete q;
      return s->error;
    }
    if (s->stop || s->inbox.size() + s->st.waiting >= s->cfg.max_queue) {
      s->st.rejected++;
      delete q;
      return PRAND_EBUSY;
    }
    q->ticket = s->next_ticket++;
    q->t_submit = s->now();
    s->inbox.push_back(q);
    s->st.submitted++;
    *ticket = q->ticket;
  }
  s->cv_work.notify_one();
  return PRAND_OK;
}

int prand_server_poll(prand_server* s, prand_completion* out, uint32_t max, uint32_t* count, int wait_ms) {
  if (!s || !count || (max && !out)) return PRAND_EINVAL;
  *count = 0;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && wait_ms > 0 && !s->error)
    s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [s] { return !s->done.empty() || s->error; });
  uint32_t k = 0;
  while (k < max && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *count = k;
  return s->error && k == 0 ? s->error : PRAND_OK;
}

int prand_server_release(prand_server* s, uint64_t ticket) {
  if (!s) return PRAND_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->finished.count(ticket)) return PRAND_EINVAL;
    s->release_q.push_back(ticket);
  }
  s->cv_work.notify_one();
  return PRAND_OK;
}

int prand_server_get_stats(prand_server* s, prand_server_stats* out) {
  if (!s || !out) return PRAND_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  return PRAND_OK;
}

double prand_server_clock(const prand_server* s) { return s ? s->now() : 0.0; }

int prand_server_destroy(prand_server* s) {
  if (!s) return PRAND_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  free_server(s);
  return PRAND_OK;
}

}  // extern "C"
