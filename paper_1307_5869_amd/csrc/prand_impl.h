// Internal declarations shared by the host side and the HIP kernels of the
// PRAND library for gfx950.  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <mutex>
#include <utility>
#include <vector>

#include "prand.h"

namespace prand {

constexpr int kMaxLimbs = 8;        // distances up to 2^512
constexpr int kLadder = 512;        // jump tables hold M^(2^b) for b < 512

// ---- state blobs (layout documented in prand.h) ----
struct MtState {
  uint32_t mt[624];
  uint32_t idx;
  uint32_t pad[3];
};
struct MrgState {
  uint32_t x[3];   // x_n, x_{n-1}, x_{n-2}
  uint32_t y[3];   // y_n, y_{n-1}, y_{n-2}
};
struct LfsrState {
  uint32_t z[4];
};
struct GmState {
  uint64_t xp[32];  // x^(n-1)
  uint64_t xc[32];  // x^(n)
  uint32_t off;     // GQ58.3: words of the current 8-step block already consumed
  uint32_t pad;
};
static_assert(sizeof(MtState) == 2512, "MT19937 state layout");
static_assert(sizeof(MrgState) == 24, "MRG32K3A state layout");
static_assert(sizeof(LfsrState) == 16, "LFSR113 state layout");
static_assert(sizeof(GmState) == 520, "GM state layout");

// ---- MRG32K3A constants: matrices A, B of the paper's MRG32K3A section ----
constexpr uint32_t kMrgM1 = 4294967087u;   // 2^32 - 209
constexpr uint32_t kMrgM2 = 4294944443u;   // 2^32 - 22853
constexpr uint32_t kMrgA12 = 1403580u;     // a
constexpr uint32_t kMrgA13n = 810728u;     // -b
constexpr uint32_t kMrgA21 = 527612u;      // c
constexpr uint32_t kMrgA23n = 1370589u;    // -d

// ---- GM/GQ parameters of the paper's Table 2 ----
// g = p * 2^t; s = ensemble size, v = digit bits per element.
struct GmParams {
  uint64_t k, q, p;
  int t, v, s;
  int n0;  // M^N = 0 mod 2^t for N >= n0 (composite moduli only)
};
constexpr GmParams kGmParams[8] = {
    /* GM19   */ {15, 28, 524287ull, 0, 1, 32, 0},
    /* GM29   */ {4, 2, 536870909ull, 0, 1, 32, 0},
    /* GM31   */ {11, 14, 2147483647ull, 0, 1, 32, 0},
    /* GM55   */ {256, 176, 2251799813685119ull, 4, 4, 8, 2},
    /* GM61   */ {24, 74, 2305843009213693951ull, 0, 1, 32, 0},
    /* GQ58.1 */ {8, 48, 536870909ull, 29, 1, 32, 16},
    /* GQ58.3 */ {8, 48, 536870909ull, 29, 3, 12, 16},
    /* GQ58.4 */ {8, 48, 536870909ull, 29, 4, 8, 16},
};
inline bool is_gm(int gen) { return gen >= PRAND_GM19 && gen <= PRAND_GQ58X4; }

// Byte tables for block splitting with each generator's default variant:
// the stream of id starts id 2^e steps on (e = kGmByteE[G], kLfsrByteE, the
// default block exponents), applied as one matrix per nonzero byte d_j of
// id (id = sum d_j 2^(8 j)): entry [j][d] is the jump by d 2^(e + 8 j), so a
// stream costs at most 8 matrix applications instead of one per set bit.
constexpr int kGmByteE[8] = {23, 27, 27, 34, 34, 27, 27, 27};
constexpr int kLfsrByteE = 34;

// ---- device-resident jump tables (built once per context) ----
struct DeviceTables {
  uint32_t* mrg = nullptr;    // [kLadder][18]: A^(2^b) mod m1 (row major), B^(2^b) mod m2
  uint32_t* lfsr = nullptr;   // [kLadder][4][32]: columns of T_c^(2^b)
  uint64_t* gm = nullptr;     // [8][kLadder][4]: (a b; c d) = M^(2^b) mod p
  uint64_t* gmbyte = nullptr;   // [8][8][256][4]: M^(d 2^(kGmByteE[G] + 8 j)) mod p
  uint64_t* gmneg = nullptr;    // [8][4]: M^(-n0) mod p (composite moduli; identity otherwise)
  uint32_t* lfsrbyte = nullptr; // [8][256][4][32]: columns of T_c^(d 2^(kLfsrByteE + 8 j))
  uint32_t* mt = nullptr;     // [kLadder][624]: bits of x^(2^b) mod phi (19937 used)
  uint32_t* mtdiglo = nullptr;  // [3][65536][624]: x^(d 2^(kMtDigitE + 16k)) mod phi
  uint32_t* mtdig8hi = nullptr; // [2][256][624]: x^(d 2^(kMtDigitE + 48 + 8j)) mod phi
  void* mttop = nullptr;        // [65536] MtState: the default state jumped t 2^(kMtDigitE + 48)
  uint32_t* mtblk = nullptr;    // [kMtBlkPolys][624]: x^(624 2^(kMtBlkFirst + i)) mod phi
  uint32_t* mtinv = nullptr;    // [624]: x^(-1) mod phi
  void* defaults = nullptr;   // default state of each generator, 11 x 2560 bytes
};
constexpr size_t kDefaultStride = 2560;
// exponent of the MT19937 digit tables: the block-splitting block 2^432
constexpr int kMtDigitE = 432;
// whole-block MT19937 jumps for batched sections of 624 2^kMtBlkFirst outputs
// (tasks up to 2^40 outputs: section numbers below 2^22)
constexpr int kMtBlkFirst = 10;
constexpr int kMtBlkPolys = 22;

// Order a wavefront's LDS writes before its later LDS reads (and reads before
// later writes) when the LDS block is private to the wavefront: LDS
// instructions of one wavefront execute in order, so only the compiler must
// be kept from reordering.  No workgroup barrier: wavefronts of one workgroup
// may run different amounts of work (or leave early).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 16-byte output store of the bulk generators.  u32/f32 outputs are marked
// non-temporal (the kernel that writes them never reads them back) when the
// caller's store instructions cover whole 128-byte lines (kLines); f64
// outputs and partial-line pieces stay plain.  Measured against plain stores, in alternation on one
// box: MT19937 u32 0.912 -> 0.861 ms per 2^30 words, LFSR113 u32 0.82 ->
// 0.81 ms, MRG32K3A within noise; in f64 non-temporal stores were slower
// (MRG32K3A and LFSR113 by 4 %, and MT19937, whose two stores per lane each
// cover half of every 32-byte piece, took twice as long).
template <int DT, bool kLines = true>
__device__ __forceinline__ void store_out16(void* p, uint4 v) {
  if (DT == PRAND_F64 || !kLines) {
    *(uint4*)p = v;
  } else {
    typedef unsigned int U4 __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(1))) U4 GU4;
    U4 w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, (GU4*)p);
  }
}

// ---- launchers (one per kernel family); all enqueue on `st` ----
// Distances: `dist` holds nlimbs limbs per stream when per_stream, else one
// shared distance.  `ids` + `block_e`: distance id * 2^block_e (GQ58.3: in
// ensemble steps).  Exactly one of (dist, ids) is used.
struct JumpSpec {
  const uint64_t* dist = nullptr;
  int nlimbs = 0;
  int per_stream = 0;
  const uint64_t* ids = nullptr;
  int block_e = 0;
  // MT19937 block splitting from the default state: the states of the top
  // 16 bits of an id (DeviceTables::mttop), or null
  const void* mt_top = nullptr;
  // MT19937, per-stream one-limb distances: counted in whole sections of
  // 624 2^kMtBlkFirst outputs (jumped by the whole-block table, one
  // polynomial per set bit, where the state sits on a block boundary and the
  // distance is below 2^kMtBlkPolys sections; otherwise through the ladder)
  int mt_blocks = 0;
};

// sectab: the section-start table of seclen, or null (ladder jumps)
hipError_t launch_mrg_generate(const DeviceTables& T, const MrgState* sin, MrgState* sout, uint32_t count,
                               uint64_t n, int nsec_log2, uint64_t seclen, int dtype, void* out,
                               const uint32_t* sectab, hipStream_t st);
hipError_t launch_mrg_jump(const DeviceTables& T, MrgState* states, uint32_t count, const JumpSpec& js,
                           const MrgState* base, hipStream_t st);

hipError_t launch_lfsr_generate(const DeviceTables& T, const LfsrState* sin, LfsrState* sout, uint32_t count,
                                uint64_t n, int nsec_log2, uint64_t seclen, int dtype, void* out,
                                const uint32_t* sectab, hipStream_t st);
hipError_t launch_lfsr_jump(const DeviceTables& T, LfsrState* states, uint32_t count, const JumpSpec& js,
                            const LfsrState* base, hipStream_t st);

hipError_t launch_mt_generate(MtState* states, uint32_t count, uint64_t n, int dtype, void* out,
                              hipStream_t st);
hipError_t launch_mt_jump(const DeviceTables& T, MtState* states, uint32_t count, const JumpSpec& js,
                          const MtState* base, hipStream_t st);

hipError_t launch_gm_generate(const DeviceTables& T, int gen, const GmState* sin, GmState* sout,
                              uint32_t count, uint64_t n, int dtype, void* out, hipStream_t st);
hipError_t launch_gm_jump(const DeviceTables& T, int gen, GmState* states, uint32_t count, const JumpSpec& js,
                          const GmState* base, hipStream_t st);

hipError_t launch_seed(int gen, const uint64_t* seeds, uint32_t count, void* states, hipStream_t st);
// the same seeding on the host (no GPU): one state blob of `gen`
void seed_host(int gen, uint64_t seed, void* h_state);

// ---- host-side table construction (context set-up) ----
struct HostTables {
  uint32_t mrg[kLadder * 18];
  uint32_t lfsr[kLadder * 4 * 32];
  uint64_t gm[8 * kLadder * 4];
  uint64_t gmbyte[8 * 8 * 256 * 4];
  uint64_t gmneg[8 * 4];
  uint32_t lfsrbyte[8 * 256 * 128];
};
void build_mrg_ladder(uint32_t* out);
void build_lfsr_ladder(uint32_t* out);
// Section-start tables of the many-stream MRG32K3A/LFSR113 kernels: for a
// section length L, row j - 1 (j = 1 .. kSectionTableRows) holds the jump by
// j L (MRG32K3A: A^(jL) mod m1 then B^(jL) mod m2, 18 words; LFSR113: the
// columns of T_c^(jL) for c = 0..3, 128 words), so section j of a stream
// starts from one matrix application instead of one per set bit of j L.
constexpr int kSectionTableRows = 63;
constexpr int kMrgSectionWords = 18;
constexpr int kLfsrSectionWords = 128;
void build_mrg_section_table(uint64_t seclen, uint32_t* out);
void build_lfsr_section_table(uint64_t seclen, uint32_t* out);
void build_gm_ladders(uint64_t* out);
void build_gm_byte_tables(uint64_t* out, uint64_t* neg);
void build_lfsr_byte_table(uint32_t* out);

// the calling thread's current device is set to `dev` for the guard's life
struct DeviceGuard {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) err = hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace prand

// the opaque context of the public ABI
struct prand_ctx {
  int device = 0;
  int num_cus = 256;
  char arch[64] = {0};
  prand::DeviceTables T;
  bool mt_ready = false;
  std::mutex mu;          // guards mt_ready, the host-call scratch and the section buffer
  void* scratch = nullptr;
  // prand_generate's section states and distances, kept between calls and
  // grown when a call needs more (freed with the context)
  void* sec_buf = nullptr;
  size_t sec_buf_bytes = 0;
  int last_hip = 0;
  // section-start tables by section length, [0] MRG32K3A, [1] LFSR113
  // (built on first use, immutable afterwards, freed with the context)
  std::mutex sec_mu;
  std::vector<std::pair<uint64_t, uint32_t*>> sec_tabs[2];
};

namespace prand {
// build and upload the MT19937 jump polynomials once per context
int ensure_mt_tables(prand_ctx* c);
// whether the MT19937 jump polynomials are built (never builds them)
bool mt_tables_ready(prand_ctx* c);
// the sectioned fill of one host state (prand_generate); with `scratch` set
// it keeps its section states there and allocates nothing
int generate_host_state(prand_ctx* c, int gen, void* h_state, int dtype, void* d_out, uint64_t n,
                        hipStream_t st, void* scratch, size_t scratch_bytes);
// once per device, with that device current: look up the device address of
// the allocation-free entry point's static array
hipError_t noalloc_setup(int device);

inline int hipfail(prand_ctx* c, hipError_t e) {
  if (c) c->last_hip = (int)e;
  return PRAND_EHIP;
}
}  // namespace prand
