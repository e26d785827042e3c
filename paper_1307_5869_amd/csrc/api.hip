// The C ABI declared in include/prand.h: argument checks, context set-up and
// the choice of launch shapes.  Every generated number and every jump is
// computed by the HIP kernels; host code here only validates, plans and
// copies states for the entry points that take host states.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "mt_poly.h"
#include "prand_impl.h"

using namespace prand;

namespace {

constexpr size_t kScratch = 64 * 1024;

bool valid_gen(int g) { return g >= 0 && g < PRAND_NUM_GENERATORS; }
bool valid_dtype(int d) { return d >= PRAND_U32 && d <= PRAND_F64; }

size_t state_bytes(int g) {
  switch (g) {
    case PRAND_MT19937: return sizeof(MtState);
    case PRAND_MRG32K3A: return sizeof(MrgState);
    case PRAND_LFSR113: return sizeof(LfsrState);
    default: return valid_gen(g) ? sizeof(GmState) : 0;
  }
}
size_t elem_bytes(int dtype) { return dtype == PRAND_F64 ? 8 : 4; }

// Block-splitting block lengths, log2 of ensemble steps, per initialising
// function of the paper's Table 4: the smallest power of two no shorter than
// the table's maximal sequence length.  -1: function not provided.
constexpr int kBlockLog2[PRAND_NUM_GENERATORS][4] = {
    /*            SEQ SHORT MEDIUM LONG */
    /* MT19937  */ {432, -1, -1, -1},
    /* MRG32K3A */ {127, -1, -1, -1},
    /* LFSR113  */ {34, -1, -1, 80},
    /* GM19     */ {23, -1, -1, -1},
    /* GM29     */ {-1, 27, 33, 40},
    /* GM31     */ {-1, 27, 33, 40},
    /* GM55     */ {-1, 34, -1, 67},
    /* GM61     */ {34, -1, -1, 85},
    /* GQ58.1   */ {-1, 27, 33, 40},
    /* GQ58.3   */ {-1, 27, 33, 40},
    /* GQ58.4   */ {-1, 27, 33, 40},
};
// Table 4: (number of sequences, maximal length) per initialising function
constexpr double kLimits[PRAND_NUM_GENERATORS][4][2] = {
    /* MT19937  */ {{1e19, 1e130}, {0, 0}, {0, 0}, {0, 0}},
    /* MRG32K3A */ {{1e19, 1e38}, {0, 0}, {0, 0}, {0, 0}},
    /* LFSR113  */ {{3.8e18, 1e10}, {0, 0}, {0, 0}, {4e9, 1e24}},
    /* GM19     */ {{1e3, 6e6}, {0, 0}, {0, 0}, {0, 0}},
    /* GM29     */ {{0, 0}, {1e8, 8e7}, {1e6, 8e9}, {1e4, 8e11}},
    /* GM31     */ {{0, 0}, {1e9, 8e7}, {1e7, 8e9}, {1e5, 8e11}},
    /* GM55     */ {{0, 0}, {1e18, 1e10}, {0, 0}, {4e9, 1e20}},
    /* GM61     */ {{1.8e19, 1e10}, {0, 0}, {0, 0}, {4e9, 3e25}},
    /* GQ58.1   */ {{0, 0}, {1e8, 8e7}, {1e6, 8e9}, {1e4, 8e11}},
    /* GQ58.3   */ {{0, 0}, {2e8, 8e7}, {2e6, 8e9}, {2e4, 8e11}},
    /* GQ58.4   */ {{0, 0}, {3e8, 8e7}, {3e6, 8e9}, {3e4, 8e11}},
};

// the byte tables are built for each generator's default block exponent
constexpr int default_block_log2(int gen) { return kBlockLog2[gen][0] >= 0 ? kBlockLog2[gen][0] : kBlockLog2[gen][1]; }
constexpr bool byte_tables_match() {
  for (int g = 0; g < 8; g++)
    if (kGmByteE[g] != default_block_log2(PRAND_GM19 + g)) return false;
  return kLfsrByteE == default_block_log2(PRAND_LFSR113);
}
static_assert(byte_tables_match(), "byte tables built for another block exponent");

// the documented default seed of each generator: MT19937 5489, MRG32K3A and
// LFSR113 12345, GM/GQ 0
uint64_t default_seed(int gen) { return gen == PRAND_MT19937 ? 5489 : (gen <= PRAND_LFSR113 ? 12345 : 0); }

int block_log2(int gen, int variant) {
  if (!valid_gen(gen) || variant < PRAND_SEQ_DEFAULT || variant > PRAND_SEQ_LONG) return PRAND_EINVAL;
  if (variant == PRAND_SEQ_DEFAULT) {
    const int e = kBlockLog2[gen][0];
    return e >= 0 ? e : kBlockLog2[gen][1];
  }
  const int e = kBlockLog2[gen][variant - 1];
  return e >= 0 ? e : PRAND_EUNSUPPORTED;
}

int resolve_variant(int gen, int variant) {
  if (variant != PRAND_SEQ_DEFAULT) return variant;
  return kBlockLog2[gen][0] >= 0 ? PRAND_SEQ : PRAND_SEQ_SHORT;
}

template <class T>
hipError_t upload(T** dst, const T* src, size_t n) {
  hipError_t e = hipMalloc((void**)dst, n * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
}

// The MT19937 tables (656 MB, read-only once built) are shared by the
// contexts of one device: the first context that needs them builds them, the
// others take references, the last one to go frees them.
struct MtTables {
  uint32_t *mt = nullptr, *mtblk = nullptr, *mtinv = nullptr, *mtdiglo = nullptr, *mtdig8hi = nullptr;
  void* mttop = nullptr;
  int refs = 0;
};
std::mutex g_mt_mu;
std::map<int, MtTables> g_mt_tables;   // by device

void take_mt_tables(prand_ctx* c, const MtTables& t) {
  c->T.mt = t.mt;
  c->T.mtblk = t.mtblk;
  c->T.mtinv = t.mtinv;
  c->T.mtdiglo = t.mtdiglo;
  c->T.mtdig8hi = t.mtdig8hi;
  c->T.mttop = t.mttop;
  c->mt_ready = true;
}

void free_mt_fields(prand_ctx* c) {
  (void)hipFree(c->T.mt);
  (void)hipFree(c->T.mtdiglo);
  (void)hipFree(c->T.mtdig8hi);
  (void)hipFree(c->T.mttop);
  (void)hipFree(c->T.mtblk);
  (void)hipFree(c->T.mtinv);
}

// a context's share of the tables goes (at destruction; its device current)
void release_mt_tables(prand_ctx* c) {
  if (!c->mt_ready) {
    free_mt_fields(c);   // what a failed build left, if anything
    return;
  }
  std::lock_guard<std::mutex> lk(g_mt_mu);
  auto it = g_mt_tables.find(c->device);
  if (it != g_mt_tables.end() && --it->second.refs == 0) {
    free_mt_fields(c);
    g_mt_tables.erase(it);
  }
}

hipError_t ensure_mt(prand_ctx* c) {
  // caller holds c->mu
  if (c->mt_ready) return hipSuccess;
  std::lock_guard<std::mutex> glk(g_mt_mu);
  {
    auto it = g_mt_tables.find(c->device);
    if (it != g_mt_tables.end()) {
      it->second.refs++;
      take_mt_tables(c, it->second);
      return hipSuccess;
    }
  }
  std::vector<uint32_t> mt((size_t)kLadder * 624), dlo((size_t)kMtLoDigits * kMtLoSize * 624),
      d8((size_t)2 * 256 * 624);
  std::vector<uint32_t> blk((size_t)kMtBlkPolys * 624), inv(624);
  if (!mt_build_polys(mt.data(), kLadder, dlo.data(), d8.data(), kMtDigitE)) return hipErrorUnknown;
  if (!mt_build_block_polys(kMtBlkFirst + kMtBlkPolys + 9, kMtBlkFirst, kMtBlkPolys, blk.data(), inv.data()))
    return hipErrorUnknown;
  hipError_t e = upload(&c->T.mt, mt.data(), mt.size());
  if (e == hipSuccess) e = upload(&c->T.mtblk, blk.data(), blk.size());
  if (e == hipSuccess) e = upload(&c->T.mtinv, inv.data(), inv.size());
  if (e == hipSuccess) e = upload(&c->T.mtdiglo, dlo.data(), dlo.size());
  if (e == hipSuccess) e = upload(&c->T.mtdig8hi, d8.data(), d8.size());
  // the default state jumped t * 2^(432 + 48) for every top-16-bit value t
  // of an id, by the jump kernel's general digit path
  uint64_t* d_ids = nullptr;
  if (e == hipSuccess) e = hipMalloc(&c->T.mttop, (size_t)65536 * sizeof(MtState));
  if (e == hipSuccess) e = hipMalloc((void**)&d_ids, 65536 * sizeof(uint64_t));
  if (e == hipSuccess) {
    std::vector<uint64_t> ids(65536);
    for (uint64_t t = 0; t < 65536; t++) ids[t] = t << 48;
    e = hipMemcpy(d_ids, ids.data(), ids.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) {
    JumpSpec js;
    js.ids = d_ids;
    js.block_e = kMtDigitE;
    e = launch_mt_jump(c->T, (MtState*)c->T.mttop, 65536, js,
                       (const MtState*)((const char*)c->T.defaults + kDefaultStride * PRAND_MT19937), nullptr);
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  (void)hipFree(d_ids);
  if (e == hipSuccess) {
    MtTables t;
    t.mt = c->T.mt;
    t.mtblk = c->T.mtblk;
    t.mtinv = c->T.mtinv;
    t.mtdiglo = c->T.mtdiglo;
    t.mtdig8hi = c->T.mtdig8hi;
    t.mttop = c->T.mttop;
    t.refs = 1;
    g_mt_tables[c->device] = t;
    c->mt_ready = true;
  }
  return e;
}

int ensure_mt_locked(prand_ctx* c, int gen) {
  if (gen != PRAND_MT19937) return PRAND_OK;
  std::lock_guard<std::mutex> lk(c->mu);
  hipError_t e = ensure_mt(c);
  return e == hipSuccess ? PRAND_OK : hipfail(c, e);
}

hipError_t launch_jump(prand_ctx* c, int gen, void* states, uint32_t count, const JumpSpec& js, const void* base,
                       hipStream_t st) {
  switch (gen) {
    case PRAND_MT19937: return launch_mt_jump(c->T, (MtState*)states, count, js, (const MtState*)base, st);
    case PRAND_MRG32K3A: return launch_mrg_jump(c->T, (MrgState*)states, count, js, (const MrgState*)base, st);
    case PRAND_LFSR113: return launch_lfsr_jump(c->T, (LfsrState*)states, count, js, (const LfsrState*)base, st);
    default: return launch_gm_jump(c->T, gen, (GmState*)states, count, js, (const GmState*)base, st);
  }
}

// The section-start table of MRG32K3A/LFSR113 (k = 0/1) for section length
// seclen: looked up, or built on the host and uploaded when `may_create`
// (an allocation and a blocking copy, once per length; not while the stream
// is being captured, and at most kMaxSectionTables lengths per generator).
// Null when there is none: the kernel then jumps through the ladder.
constexpr size_t kMaxSectionTables = 64;

const uint32_t* section_table(prand_ctx* c, int k, uint64_t seclen, hipStream_t st, bool may_create) {
  std::lock_guard<std::mutex> lk(c->sec_mu);
  for (const auto& t : c->sec_tabs[k])
    if (t.first == seclen) return t.second;
  if (!may_create || c->sec_tabs[k].size() >= kMaxSectionTables) return nullptr;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
  const size_t words = (size_t)kSectionTableRows * (k == 0 ? kMrgSectionWords : kLfsrSectionWords);
  std::vector<uint32_t> h(words);
  if (k == 0) build_mrg_section_table(seclen, h.data());
  else build_lfsr_section_table(seclen, h.data());
  uint32_t* d = nullptr;
  if (hipMalloc((void**)&d, words * 4) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (hipMemcpy(d, h.data(), words * 4, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(d);
    return nullptr;
  }
  c->sec_tabs[k].push_back({seclen, d});
  return d;
}

// sections per stream (log2) and section length of the many-stream
// MRG32K3A/LFSR113 kernel: up to 64 sections per stream, section starts
// 16-byte aligned.  With a section-start table a start costs one matrix
// application, so streams are cut into as many sections of at least 256
// outputs as fit in 2^22 lanes (more, shorter sections measured faster: the
// 64 runs of a wavefront then lie close together in the output); with ladder
// jumps a start costs one application per set bit of its distance, so the
// cut stops at 2^19 lanes and sections of at least 64 outputs.
void section_plan(uint32_t count, uint64_t n, bool table, int& nsec_log2, uint64_t& seclen) {
  nsec_log2 = 0;
  if (table) {
    while (nsec_log2 < 6 && ((uint64_t)count << (nsec_log2 + 1)) <= (1ull << 22) && (n >> (nsec_log2 + 1)) >= 256)
      nsec_log2++;
  } else {
    while (nsec_log2 < 6 && ((uint64_t)count << nsec_log2) < (1ull << 19) && (n >> (nsec_log2 + 1)) >= 64)
      nsec_log2++;
  }
  seclen = (n + (1ull << nsec_log2) - 1) >> nsec_log2;
  seclen = (seclen + 3) & ~3ull;
  if (seclen == 0) seclen = 4;
}

// many-stream generation; sin/sout may alias (sections of a stream never
// straddle a wavefront).  may_alloc: a section-start table may be built.
hipError_t launch_streams(prand_ctx* c, int gen, const void* sin, void* sout, uint32_t count, uint64_t n,
                          int dtype, void* out, hipStream_t st, bool may_alloc) {
  if (gen == PRAND_MRG32K3A || gen == PRAND_LFSR113) {
    const int k = gen == PRAND_MRG32K3A ? 0 : 1;
    int nsec_log2;
    uint64_t seclen;
    section_plan(count, n, true, nsec_log2, seclen);
    const uint32_t* tab = nsec_log2 ? section_table(c, k, seclen, st, may_alloc) : nullptr;
    if (!tab) section_plan(count, n, false, nsec_log2, seclen);
    if (gen == PRAND_MRG32K3A)
      return launch_mrg_generate(c->T, (const MrgState*)sin, (MrgState*)sout, count, n, nsec_log2, seclen, dtype,
                                 out, tab, st);
    return launch_lfsr_generate(c->T, (const LfsrState*)sin, (LfsrState*)sout, count, n, nsec_log2, seclen, dtype,
                                out, tab, st);
  }
  if (gen == PRAND_MT19937) {
    if (sin != sout) {
      hipError_t e = hipMemcpyAsync(sout, sin, (size_t)count * sizeof(MtState), hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return e;
    }
    return launch_mt_generate((MtState*)sout, count, n, dtype, out, st);
  }
  return launch_gm_generate(c->T, gen, (const GmState*)sin, (GmState*)sout, count, n, dtype, out, st);
}

// distances of the section starts: j * seclen for the bulk sections j < nb,
// then T for the final section
__global__ void section_dist_kernel(uint64_t* d, uint32_t nb, uint64_t seclen, uint64_t T) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb) d[i] = (uint64_t)i * seclen;
  else if (i == nb) d[i] = T;
}

}  // namespace

int prand::ensure_mt_tables(prand_ctx* c) {
  DeviceGuard g(c->device);
  return ensure_mt_locked(c, PRAND_MT19937);
}

// The sectioned fill behind prand_generate and prand_generate_noalloc.
// Bulk sections of 2^k outputs cover [0, T); each starts from the state
// jumped j * 2^k ahead (one ladder application per set bit of j) and fills
// its slice.  A final section covers [T, n) and leaves the advanced state.
// For MT19937, T is the last twist-block boundary of the original stream
// before n: a jump yields the canonical window, which differs from the array
// sequential generation holds only in bits the next twist overwrites, so the
// final section's state is exactly the sequential one.  The section states,
// their distances and the copied-in base state live in `scratch` when it is
// given (the plan then uses at most as many sections as fit in
// scratch_bytes; the output does not depend on the plan), else in memory
// allocated for the call.  Arguments are checked by the caller; MT19937
// tables must exist.
int prand::generate_host_state(prand_ctx* c, int gen, void* h_state, int dtype, void* d_out, uint64_t n,
                               hipStream_t st, void* scratch, size_t scratch_bytes) {
  uint64_t min_sec, max_secs;
  switch (gen) {
    case PRAND_MT19937: min_sec = 1ull << 18; max_secs = 4096; break;
    case PRAND_MRG32K3A:
    case PRAND_LFSR113: min_sec = 256; max_secs = 1u << 19; break;
    default: min_sec = 4096; max_secs = 1u << 16; break;
  }
  const size_t sb = state_bytes(gen);
  const size_t es = elem_bytes(dtype);
  const size_t base_bytes = (sb + 255) & ~(size_t)255;
  if (scratch) {
    // base state, then distances, then states, each 256-byte aligned
    if (scratch_bytes < base_bytes + 2 * 256 + 2 * (sb + 8)) return PRAND_ERANGE;
    const uint64_t fit = (scratch_bytes - base_bytes - 2 * 256) / (sb + 8);   // section states that fit
    max_secs = std::min<uint64_t>(max_secs, fit - 1);
  }
  int k = 0;
  while ((1ull << k) < min_sec) k++;
  while (((n + (1ull << k) - 1) >> k) > max_secs) k++;
  const bool one = (1ull << k) >= n;
  const uint64_t seclen = one ? n : (1ull << k);
  uint64_t T;
  if (one) {
    T = 0;
  } else if (gen == PRAND_MT19937) {
    const uint32_t idx0 = std::min<uint32_t>(((const MtState*)h_state)->idx, 624u);
    const uint64_t r0 = 624 - idx0;
    T = (n <= r0) ? 0 : r0 + 624 * ((n - r0 + 623) / 624 - 1);
  } else {
    T = ((n + seclen - 1) / seclen - 1) * seclen;
  }
  const uint64_t full = T / seclen, part = T % seclen;
  const uint64_t nb = full + (part ? 1 : 0);   // bulk sections
  const uint64_t nst = nb + 1;                 // plus the final one
  void* d_states = nullptr;
  uint64_t* d_dist = nullptr;
  void* d_base = nullptr;
  hipError_t e = hipSuccess;
  std::unique_lock<std::mutex> lk(c->mu, std::defer_lock);
  if (scratch) {
    const size_t dist_off = base_bytes;
    const size_t st_off = dist_off + ((nst * 8 + 255) & ~(size_t)255);
    if (st_off + nst * sb > scratch_bytes) return PRAND_ERANGE;
    d_base = scratch;
    d_dist = (uint64_t*)((char*)scratch + dist_off);
    d_states = (char*)scratch + st_off;
  } else {
    // the context's host-call scratch holds the base state; its section
    // buffer (grown when too small, otherwise reused: no allocation and no
    // implicit device synchronisation per call) the distances and states
    lk.lock();
    d_base = c->scratch;
    const size_t st_off = (nst * 8 + 255) & ~(size_t)255;
    const size_t need = st_off + nst * sb;
    if (need > c->sec_buf_bytes) {
      (void)hipFree(c->sec_buf);
      c->sec_buf = nullptr;
      c->sec_buf_bytes = 0;
      e = hipMalloc(&c->sec_buf, need);
      if (e == hipSuccess) c->sec_buf_bytes = need;
    }
    if (e == hipSuccess) {
      d_dist = (uint64_t*)c->sec_buf;
      d_states = (char*)c->sec_buf + st_off;
    }
  }
  if (e == hipSuccess) e = hipMemcpyAsync(d_base, h_state, sb, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(section_dist_kernel, dim3((uint32_t)((nst + 255) / 256)), dim3(256), 0, st, d_dist,
                       (uint32_t)nb, seclen, T);
    e = hipGetLastError();
  }
  JumpSpec js;
  js.dist = d_dist;
  js.nlimbs = 1;
  js.per_stream = 1;
  if (e == hipSuccess) e = launch_jump(c, gen, d_states, (uint32_t)nst, js, d_base, st);
  if (e == hipSuccess && full)
    e = launch_streams(c, gen, d_states, d_states, (uint32_t)full, seclen, dtype, d_out, st, !scratch);
  if (e == hipSuccess && part) {
    void* sp = (char*)d_states + full * sb;
    e = launch_streams(c, gen, sp, sp, 1, part, dtype, (char*)d_out + full * seclen * es, st, !scratch);
  }
  void* last = (char*)d_states + nb * sb;
  if (e == hipSuccess)
    e = launch_streams(c, gen, last, last, 1, n - T, dtype, (char*)d_out + T * es, st, !scratch);
  if (e == hipSuccess) e = hipMemcpyAsync(h_state, last, sb, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e == hipSuccess ? PRAND_OK : hipfail(c, e);
}

bool prand::mt_tables_ready(prand_ctx* c) {
  std::lock_guard<std::mutex> lk(c->mu);
  return c->mt_ready;
}

extern "C" {

const char* prand_strerror(int code) {
  switch (code) {
    case PRAND_OK: return "success";
    case PRAND_EINVAL: return "invalid argument";
    case PRAND_EUNSUPPORTED: return "variant not provided for this generator";
    case PRAND_ERANGE: return "size out of range";
    case PRAND_EHIP: return "HIP runtime error";
    case PRAND_ENOMEM: return "out of memory";
    case PRAND_ENODEV: return "no usable gfx950 device";
    case PRAND_EBUSY: return "request queue full";
    case PRAND_ENOTREADY: return "context tables this call needs are not built yet";
    default: return "unknown error";
  }
}

int prand_last_hip_error(const prand_ctx* ctx) { return ctx ? ctx->last_hip : 0; }

size_t prand_state_bytes(int gen) { return state_bytes(gen); }

int prand_block_log2(int gen, int variant) { return block_log2(gen, variant); }

int prand_independence_limit(int gen, int variant, double* max_streams, double* max_length) {
  const int e = block_log2(gen, variant);
  if (e < 0) return e;
  if (!max_streams || !max_length) return PRAND_EINVAL;
  const int v = resolve_variant(gen, variant) - 1;
  *max_streams = kLimits[gen][v][0];
  *max_length = kLimits[gen][v][1];
  return PRAND_OK;
}

int prand_ctx_create(prand_ctx** out, int hip_device) {
  if (!out) return PRAND_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) return PRAND_ENODEV;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return PRAND_ENODEV;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return PRAND_ENODEV;
  DeviceGuard g(hip_device);
  if (g.err != hipSuccess) return PRAND_ENODEV;
  prand_ctx* c = new (std::nothrow) prand_ctx;
  if (!c) return PRAND_ENOMEM;
  c->device = hip_device;
  c->num_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  std::strncpy(c->arch, prop.gcnArchName, sizeof(c->arch) - 1);
  HostTables* H = new (std::nothrow) HostTables;
  if (!H) { delete c; return PRAND_ENOMEM; }
  build_mrg_ladder(H->mrg);
  build_lfsr_ladder(H->lfsr);
  build_gm_ladders(H->gm);
  build_gm_byte_tables(H->gmbyte, H->gmneg);
  build_lfsr_byte_table(H->lfsrbyte);
  hipError_t e = upload(&c->T.mrg, H->mrg, sizeof(H->mrg) / sizeof(H->mrg[0]));
  if (e == hipSuccess) e = upload(&c->T.lfsr, H->lfsr, sizeof(H->lfsr) / sizeof(H->lfsr[0]));
  if (e == hipSuccess) e = upload(&c->T.gm, H->gm, sizeof(H->gm) / sizeof(H->gm[0]));
  if (e == hipSuccess) e = upload(&c->T.gmbyte, H->gmbyte, sizeof(H->gmbyte) / sizeof(H->gmbyte[0]));
  if (e == hipSuccess) e = upload(&c->T.gmneg, H->gmneg, sizeof(H->gmneg) / sizeof(H->gmneg[0]));
  if (e == hipSuccess) e = upload(&c->T.lfsrbyte, H->lfsrbyte, sizeof(H->lfsrbyte) / sizeof(H->lfsrbyte[0]));
  delete H;
  if (e == hipSuccess) e = hipMalloc(&c->T.defaults, kDefaultStride * PRAND_NUM_GENERATORS);
  if (e == hipSuccess) e = hipMalloc(&c->scratch, kScratch);
  if (e == hipSuccess) e = noalloc_setup(hip_device);
  if (e == hipSuccess) {
    // default states: the documented default seed of each generator
    uint64_t seeds[PRAND_NUM_GENERATORS];
    for (int gidx = 0; gidx < PRAND_NUM_GENERATORS; gidx++)
      seeds[gidx] = default_seed(gidx);
    e = hipMemcpy(c->scratch, seeds, sizeof seeds, hipMemcpyHostToDevice);
    for (int gidx = 0; gidx < PRAND_NUM_GENERATORS && e == hipSuccess; gidx++)
      e = launch_seed(gidx, (const uint64_t*)c->scratch + gidx, 1, (char*)c->T.defaults + kDefaultStride * gidx,
                      nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
  }
  if (e != hipSuccess) {
    prand_ctx_destroy(c);
    return PRAND_EHIP;
  }
  *out = c;
  return PRAND_OK;
}

int prand_ctx_destroy(prand_ctx* c) {
  if (!c) return PRAND_OK;
  DeviceGuard g(c->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(c->T.mrg);
  (void)hipFree(c->T.lfsr);
  (void)hipFree(c->T.gm);
  (void)hipFree(c->T.gmbyte);
  (void)hipFree(c->T.gmneg);
  (void)hipFree(c->T.lfsrbyte);
  release_mt_tables(c);
  (void)hipFree(c->T.defaults);
  (void)hipFree(c->scratch);
  (void)hipFree(c->sec_buf);
  for (auto& v : c->sec_tabs)
    for (auto& t : v) (void)hipFree(t.second);
  delete c;
  return PRAND_OK;
}

int prand_seed_dev(prand_ctx* c, int gen, const uint64_t* d_seeds, uint32_t count, void* d_states, void* stream) {
  if (!c || !valid_gen(gen)) return PRAND_EINVAL;
  if (count == 0) return PRAND_OK;
  if (!d_seeds || !d_states) return PRAND_EINVAL;
  DeviceGuard g(c->device);
  hipError_t e = launch_seed(gen, d_seeds, count, d_states, (hipStream_t)stream);
  return e == hipSuccess ? PRAND_OK : hipfail(c, e);
}

int prand_seed(prand_ctx* c, int gen, uint64_t seed, void* h_state) {
  if (!c || !valid_gen(gen) || !h_state) return PRAND_EINVAL;
  DeviceGuard g(c->device);
  std::lock_guard<std::mutex> lk(c->mu);
  uint64_t* d_seed = (uint64_t*)c->scratch;
  void* d_state = (char*)c->scratch + 256;
  hipError_t e = hipMemcpy(d_seed, &seed, 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_seed(gen, d_seed, 1, d_state, nullptr);
  if (e == hipSuccess) e = hipMemcpy(h_state, d_state, state_bytes(gen), hipMemcpyDeviceToHost);
  return e == hipSuccess ? PRAND_OK : hipfail(c, e);
}

int prand_seed_host(int gen, uint64_t seed, void* h_state) {
  if (!valid_gen(gen) || !h_state) return PRAND_EINVAL;
  seed_host(gen, seed, h_state);
  return PRAND_OK;
}

int prand_init_default_host(int gen, void* h_state) {
  if (!valid_gen(gen) || !h_state) return PRAND_EINVAL;
  seed_host(gen, default_seed(gen), h_state);
  return PRAND_OK;
}

int prand_init_default(prand_ctx* c, int gen, void* h_state) {
  if (!c || !valid_gen(gen) || !h_state) return PRAND_EINVAL;
  DeviceGuard g(c->device);
  hipError_t e = hipMemcpy(h_state, (char*)c->T.defaults + kDefaultStride * gen, state_bytes(gen),
                           hipMemcpyDeviceToHost);
  return e == hipSuccess ? PRAND_OK : hipfail(c, e);
}

// Not in the public header (a test hook): jumps `count` MT19937 states by
// d_sections[i] whole sections of 624 * 2^kMtBlkFirst outputs each, the way
// the serving loop starts its sections (the whole-block table from a block
// boundary and below 2^kMtBlkPolys sections, the ladder otherwise).
int prand_internal_mt_jump_sections(prand_ctx* c, void* d_states, uint32_t count, const uint64_t* d_sections,
                                    void* stream) {
  if (!c) return PRAND_EINVAL;
  if (count == 0) return PRAND_OK;
  if (!d_states || !d_sections) return PRAND_EINVAL;
  DeviceGuard g(c->device);
  int rc = ensure_mt_locked(c, PRAND_MT19937);
  if (rc) return rc;
  JumpSpec js;
  js.dist = d_sections;
  js.nlimbs = 1;
  js.per_stream = 1;
  js.mt_blocks = 1;
  hipError_t e = launch_mt_jump(c->T, (MtState*)d_states, count, js, nullptr, (hipStream_t)stream);
  return e == hipSuccess ? PRAND_OK : hipfail(c, e);
}

int prand_skipahead_dev(prand_ctx* c, int gen, void* d_states, uint32_t count, const uint64_t* d_dist, int nlimbs,
                        int per_stream, void* stream) {
  if (!c || !valid_gen(gen) || nlimbs < 0 || nlimbs > kMaxLimbs) return PRAND_EINVAL;
  if (count == 0 || nlimbs == 0) return PRAND_OK;
  if (!d_states || !d_dist) return PRAND_EINVAL;
  DeviceGuard g(c->device);
  int rc = ensure_mt_locked(c, gen);
  if (rc) return rc;
  JumpSpec js;
  js.dist = d_dist;
  js.nlimbs = nlimbs;
  js.per_stream = per_stream ? 1 : 0;
  hipError_t e = launch_jump(c, gen, d_states, count, js, nullptr, (hipStream_t)stream);
  return e == hipSuccess ? PRAND_OK : hipfail(c, e);
}

int prand_skipahead(prand_ctx* c, int gen, void* h_state, const uint64_t* h_dist, int nlimbs) {
  if (!c || !valid_gen(gen) || !h_state || nlimbs < 0 || nlimbs > kMaxLimbs || (nlimbs > 0 && !h_dist))
    return PRAND_EINVAL;
  if (nlimbs == 0) return PRAND_OK;
  DeviceGuard g(c->device);
  int rc = ensure_mt_locked(c, gen);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  uint64_t* d_dist = (uint64_t*)c->scratch;
  void* d_state = (char*)c->scratch + 256;
  hipError_t e = hipMemcpy(d_dist, h_dist, 8 * (size_t)nlimbs, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_state, h_state, state_bytes(gen), hipMemcpyHostToDevice);
  JumpSpec js;
  js.dist = d_dist;
  js.nlimbs = nlimbs;
  if (e == hipSuccess) e = launch_jump(c, gen, d_state, 1, js, nullptr, nullptr);
  if (e == hipSuccess) e = hipMemcpy(h_state, d_state, state_bytes(gen), hipMemcpyDeviceToHost);
  return e == hipSuccess ? PRAND_OK : hipfail(c, e);
}

int prand_init_streams_dev(prand_ctx* c, int gen, int variant, const void* d_base_state, const uint64_t* d_ids,
                           uint32_t count, void* d_states, void* stream) {
  if (!c || !valid_gen(gen)) return PRAND_EINVAL;
  const int be = block_log2(gen, variant);
  if (be < 0) return be;
  if (count == 0) return PRAND_OK;
  if (!d_ids || !d_states) return PRAND_EINVAL;
  DeviceGuard g(c->device);
  int rc = ensure_mt_locked(c, gen);
  if (rc) return rc;
  JumpSpec js;
  js.ids = d_ids;
  js.block_e = be;
  const void* base = d_base_state ? d_base_state : (const char*)c->T.defaults + kDefaultStride * gen;
  if (!d_base_state && gen == PRAND_MT19937) js.mt_top = c->T.mttop;
  hipError_t e = launch_jump(c, gen, d_states, count, js, base, (hipStream_t)stream);
  return e == hipSuccess ? PRAND_OK : hipfail(c, e);
}

int prand_init_stream(prand_ctx* c, int gen, int variant, uint64_t id, void* h_state) {
  if (!c || !valid_gen(gen) || !h_state) return PRAND_EINVAL;
  const int be = block_log2(gen, variant);
  if (be < 0) return be;
  DeviceGuard g(c->device);
  int rc = ensure_mt_locked(c, gen);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  uint64_t* d_id = (uint64_t*)c->scratch;
  void* d_state = (char*)c->scratch + 256;
  hipError_t e = hipMemcpy(d_id, &id, 8, hipMemcpyHostToDevice);
  JumpSpec js;
  js.ids = d_id;
  js.block_e = be;
  if (gen == PRAND_MT19937) js.mt_top = c->T.mttop;
  if (e == hipSuccess)
    e = launch_jump(c, gen, d_state, 1, js, (const char*)c->T.defaults + kDefaultStride * gen, nullptr);
  if (e == hipSuccess) e = hipMemcpy(h_state, d_state, state_bytes(gen), hipMemcpyDeviceToHost);
  return e == hipSuccess ? PRAND_OK : hipfail(c, e);
}

int prand_generate_array(prand_ctx* c, int gen, void* h_state, int dtype, void* h_out, uint64_t n) {
  if (!c || !valid_gen(gen) || !valid_dtype(dtype) || !h_state) return PRAND_EINVAL;
  if (n == 0) return PRAND_OK;
  if (!h_out) return PRAND_EINVAL;
  if (n > (1ull << 40)) return PRAND_ERANGE;
  DeviceGuard g(c->device);
  int rc = ensure_mt_locked(c, gen);
  if (rc) return rc;
  // chunks of at most 2^26 values: each is filled on the device by the
  // sectioned fill (which continues the host state) and copied to the host
  const size_t es = elem_bytes(dtype);
  const uint64_t chunk = std::min<uint64_t>(n, 1ull << 26);
  void* d_buf = nullptr;
  hipError_t e = hipMalloc(&d_buf, chunk * es);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? PRAND_ENOMEM : hipfail(c, e);
  }
  for (uint64_t done = 0; done < n && rc == PRAND_OK; done += chunk) {
    const uint64_t m = std::min(chunk, n - done);
    rc = generate_host_state(c, gen, h_state, dtype, d_buf, m, nullptr, nullptr, 0);
    if (rc == PRAND_OK) {
      e = hipMemcpy((char*)h_out + done * es, d_buf, m * es, hipMemcpyDeviceToHost);
      if (e != hipSuccess) rc = hipfail(c, e);
    }
  }
  (void)hipFree(d_buf);
  return rc;
}

int prand_generate_streams(prand_ctx* c, int gen, void* d_states, uint32_t count, uint64_t n, int dtype,
                           void* d_out, void* stream) {
  if (!c || !valid_gen(gen) || !valid_dtype(dtype)) return PRAND_EINVAL;
  if (count == 0 || n == 0) return PRAND_OK;
  if (!d_states || !d_out) return PRAND_EINVAL;
  if (n > (1ull << 40) || (unsigned __int128)count * n * elem_bytes(dtype) > ((unsigned __int128)1 << 50))
    return PRAND_ERANGE;
  DeviceGuard g(c->device);
  hipError_t e = launch_streams(c, gen, d_states, d_states, count, n, dtype, d_out, (hipStream_t)stream, true);
  return e == hipSuccess ? PRAND_OK : hipfail(c, e);
}

int prand_generate(prand_ctx* c, int gen, void* h_state, int dtype, void* d_out, uint64_t n, void* stream) {
  if (!c || !valid_gen(gen) || !valid_dtype(dtype) || !h_state) return PRAND_EINVAL;
  if (n == 0) return PRAND_OK;
  if (!d_out) return PRAND_EINVAL;
  if (n > (1ull << 40)) return PRAND_ERANGE;
  DeviceGuard g(c->device);
  int rc = ensure_mt_locked(c, gen);
  if (rc) return rc;
  return generate_host_state(c, gen, h_state, dtype, d_out, n, (hipStream_t)stream, nullptr, 0);
}

}  // extern "C"
