// MT19937 on gfx950.
//
// Generation: one wavefront per stream, the 624-word state in LDS.  A twist
// renews the block in three dependency phases (words 0..226 read old words
// 397..623; 227..453 read words renewed in phase one; 454..623 read phase two
// and word 0), each phase parallel across the 64 lanes; whole blocks are
// written out two at a time from LDS as 16-byte pieces (dev_mt.h).
//
// Jump-ahead (paper, section on MT19937 jump-ahead, equation g_v):
// A^v Y = g_v(A) Y = sum_i a_i A^(i-1) Y with g_v = x^v mod phi.  A^(i-1) Y is
// the window of 624 consecutive raw words starting i-1 words later, so word t
// of the result is the XOR of seq[i + t] over the set coefficients i, seq
// being the raw-word sequence continued from the state.  A distance is applied
// as one polynomial x^(2^b) mod phi (from the context ladder) per set bit b;
// block splitting by id * 2^432 from a block-aligned state uses the context's
// digit tables x^(d 2^(432 + position)) mod phi instead: three 16-bit digits
// for the low 48 bits of the id and two bytes for the top 16 bits; from the
// default state the top 16 bits come from a table of precomputed states, so a
// stream costs at most 3 polynomials.
// One wavefront does one stream: the sequence is produced 227 words at a time
// into an LDS ring, and lane l accumulates outputs t = 10l .. 10l+9 while a
// register window of 10 sequence words slides over the coefficients, so each
// coefficient costs one LDS read per lane and set coefficients cost 10
// three-input XORs per two.  Launches of few streams (stream starts served
// one request at a time) give each stream a workgroup of 12 or 8 wavefronts
// that scan separate coefficient ranges and XOR their partial windows.
#include "dev_mt.h"
#include "mt_poly.h"
#include "prand_batch.h"

namespace prand {
namespace {

using namespace mt;


// Workgroup b (one wavefront) takes stream (b % 8) * (G / 8) + b / 8 for
// b < 8 (G / 8), G = count, else stream b: consecutive workgroups go to the
// eight XCDs in turn, so each XCD's L2 writes one contiguous eighth of the
// output (measured about 2 % faster than stream b).
template <int DT>
__global__ void __launch_bounds__(64) mt_generate_kernel(MtState* states, uint32_t count, uint64_t n,
                                                         void* __restrict__ out) {
  __shared__ __align__(16) uint32_t mt[2 * 624];
  const uint32_t b = blockIdx.x, per = count / 8;
  const uint32_t s = b < 8 * per ? (b % 8) * per + b / 8 : b;
  if (s >= count) return;
  constexpr int es = (DT == PRAND_F64) ? 8 : 4;
  gen_wave<DT, true>(mt, states + s, states + s, n, (char*)out + (uint64_t)s * n * es);
}

// ------------------------------------------------------------------ jump
// Launches of few streams jump each stream with several wavefronts (12 up to
// 512 streams, 8 up to 2048; one-stream starts from the default state measured
// 0.27 and 0.31 ms against 1.28 ms with one wavefront; at 4096 streams the
// ranges' repeated recurrence runs cost more than the shorter chains save).
constexpr uint32_t kMtSplit12MaxCount = 512;
constexpr uint32_t kMtSplit8MaxCount = 2048;
constexpr int kRing = 1024;                 // LDS ring of sequence words (< 900 live at a time)
constexpr int kMask = kRing - 1;
constexpr int kMirror = 16;                 // ring[0..15] repeated after the end
constexpr int kDeg = 19937;
constexpr int kSeqLen = kDeg - 1 + 624;     // words seq[0..20559] take part
constexpr int kPer = 10;                    // outputs per lane: 64 * 10 >= 624

// s_waitcnt lgkmcnt(3), the other counters left at their maximum (gfx9
// encoding: vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).
__device__ __forceinline__ void wait_lds_but3() { __builtin_amdgcn_s_waitcnt(0xC37F); }

// Extend the ring to hold seq[0..upto) (227 words per phase).  Words landing
// in the first kMirror slots are also written after the ring's end, so that
// kPer consecutive words can be read from any slot without wrapping.  The
// ring belongs to one wavefront.  kBatched: a phase reads only words of
// earlier phases (j - 227 and below), so all its reads are issued before its
// writes, one LDS latency per phase; it takes 12 more registers, so it is
// used where no scan registers are live (the run up to a range's start).
template <bool kBatched>
__device__ __forceinline__ void extend(uint32_t* ring, int& gen_hi, int upto, int lane) {
  if (upto > kSeqLen) upto = kSeqLen;
  while (gen_hi < upto) {
    const int g0 = gen_hi;
    const int g1 = (g0 + 227 < kSeqLen) ? g0 + 227 : kSeqLen;
    if constexpr (kBatched) {
      uint32_t x0[4], x1[4], xm[4];
#pragma unroll
      for (int k = 0; k < 4; k++) {
        const int j = g0 + lane + 64 * k;
        if (j < g1) {
          x0[k] = ring[(j - 624) & kMask];
          x1[k] = ring[(j - 623) & kMask];
          xm[k] = ring[(j - 227) & kMask];
        }
      }
      asm volatile("" ::: "memory");
#pragma unroll
      for (int k = 0; k < 4; k++) {
        const int j = g0 + lane + 64 * k;
        if (j < g1) {
          const uint32_t v = recur(x0[k], x1[k], xm[k]);
          const int slot = j & kMask;
          ring[slot] = v;
          if (slot < kMirror) ring[slot + kRing] = v;
        }
      }
    } else {
      for (int j = g0 + lane; j < g1; j += 64) {
        const uint32_t v = recur(ring[(j - 624) & kMask], ring[(j - 623) & kMask], ring[(j - 227) & kMask]);
        const int slot = j & kMask;
        ring[slot] = v;
        if (slot < kMirror) ring[slot + kRing] = v;
      }
    }
    wave_lds_sync();
    gen_hi = g1;
  }
}

// ring[0..623] holds a window (next output = tempered successor); apply_poly
// replaces it by g(A) applied to it, g = poly (624 words of coefficient bits,
// reduced: no bit at or above 19937 is set).  Lane l accumulates outputs
// t = 10 l + r.  For the coefficients i0 .. i0 + 9 of a group it holds the
// sequence words seq[i0 + 10 l + k] (cur) and seq[i0 + 10 + 10 l + k] (nxt),
// k < 10: coefficient i0 + u adds seq[i0 + u + 10 l + r], which is
// cur[u + r] or nxt[u + r - 10].  Three register windows rotate over the
// groups: while a group runs, the window the group after next starts with
// is read from LDS (pf), so no group waits for its own LDS reads.
//
// The coefficient bits are uniform across the wavefront, so the scan over
// them is scalar branching.  Each bit is tested once; a set bit waits for the
// next set bit of its group and the two are added with one three-input XOR
// (gfx950 v_bitop3_b32, truth table 0x96) per output word: a group with c set
// coefficients costs ceil(c / 2) instead of c vector instructions per output
// word.  The scan is a chain of labels joined by gotos (mt_pairs.inc; after a
// pair the remaining nothing-pending tests are repeated in place, one taken
// branch less per pair), built with the structurizer told to leave uniform
// regions alone, so every test is one scalar compare and branch.
template <int kOff>
__device__ __forceinline__ void group(uint32_t* ring, uint32_t i0, uint32_t lo, uint32_t hi, int lane,
                                      uint32_t (&acc)[kPer],
                                      const uint32_t (&cur)[kPer], const uint32_t (&nxt)[kPer],
                                      uint32_t (&pf)[kPer]) {
  // i0 + 20 + 10 lane is even, so the window is read in 8-byte pairs
  const uint32_t* src = ring + ((i0 + 2 * kPer + kPer * lane) & (kMask & ~1));   // + k < kRing + kMirror
#pragma unroll
  for (int k = 0; k < kPer; k++) pf[k] = src[k];
  // the window nxt was read by the previous group: wait for those reads once
  // here (the three just issued may stay in flight), not before every pair
  wait_lds_but3();
#define MT_W2(k) (((k) < kPer) ? cur[(k)] : nxt[(k) - kPer])
#define MT_BIT(u) (((kOff + (u)) < 32 ? (lo >> ((kOff + (u)) & 31)) : (hi >> ((kOff + (u)) & 31))) & 1u)
#define MT_PAIR(p, q)                                                                              \
  _Pragma("unroll") for (int r = 0; r < kPer; r++) acc[r] =                                        \
      __builtin_amdgcn_bitop3_b32(acc[r], MT_W2((p) + r), MT_W2((q) + r), 0x96);
#define MT_ONE(p) _Pragma("unroll") for (int r = 0; r < kPer; r++) acc[r] ^= MT_W2((p) + r);
#include "mt_pairs.inc"
#undef MT_ONE
#undef MT_PAIR
#undef MT_BIT
#undef MT_W2
}

// Coefficients are scanned 60 at a time (six groups), each group testing its
// bits at fixed positions of two 32-bit scalar words (bits i1 .. i1 + 63).
// The three polynomial words a step needs are read one step ahead through
// the vector memory path, as a 624-word raw buffer (the byte offset in a
// vector register, so the hardware range check covers it: a word past the
// polynomial reads as zero), then moved to scalar registers.  Scalar loads
// would share the LDS wait counter and, returning out of order, force a full
// wait before every pair of a step.  Measured 3.4 % faster than scalar loads
// with masked group bits.  Also measured: the next window moved across lanes
// by DPP wavefront shifts, with only the last lane reading the ring, 4 %
// slower; the LDS reads are not the limit, the chain of scalar tests and
// branches of each wavefront is.
constexpr uint32_t kStep = 6 * kPer;
constexpr int kStepReach = 720;   // a step at i1 reads sequence words below i1 + 710

typedef __amdgpu_buffer_rsrc_t PolyBuf;

__device__ __forceinline__ PolyBuf poly_buffer(const uint32_t* poly) {
  // gfx9 buffer descriptor: base, no stride, 624 * 4 bytes, 32-bit data format
  return __builtin_amdgcn_make_buffer_rsrc((void*)poly, 0, 624 * 4, 0x00020000);
}

__device__ __forceinline__ uint32_t poly_word(PolyBuf pb, uint32_t w) {
  uint32_t off = w * 4u;
  asm volatile("" : "+v"(off));   // the whole offset in the vector operand
  return __builtin_amdgcn_raw_buffer_load_b32(pb, off, 0, 0);
}

// The sum over the coefficients c0 <= i < c1 of poly into acc (lane l holds
// outputs t = 10 l + r) for the window ring[0..623]; c0 a multiple of kStep,
// c1 one too or kDeg.  The ring is extended as far as the range needs; a
// range that starts later first runs the recurrence up to it.
__device__ __forceinline__ void scan_range(uint32_t* ring, const uint32_t* __restrict__ poly, int lane, uint32_t c0,
                                           uint32_t c1, uint32_t (&sum)[kPer]) {
  uint32_t acc[kPer];   // local: the groups' code is built on a register array
  int gen_hi = 624;
  extend<true>(ring, gen_hi, (int)c0 + kStepReach, lane);
  uint32_t wa[kPer], wb[kPer], wc[kPer];
  // the first two windows, read as group() reads the later ones (an even
  // slot; words past the ring's end are in its mirror)
  const uint32_t* w0 = ring + ((c0 + kPer * lane) & (kMask & ~1));
  const uint32_t* w1 = ring + ((c0 + kPer + kPer * lane) & (kMask & ~1));
#pragma unroll
  for (int r = 0; r < kPer; r++) {
    acc[r] = 0;
    wa[r] = w0[r];
    wb[r] = w1[r];
  }
  // bits i1 .. i1 + 59 lie in the words i1 / 32 .. i1 / 32 + 2 (the last
  // step's third word is past the polynomial and reads as zero).  The ring
  // is extended 227 words at a time and every step that its words allow runs
  // before the next extension (near the end the sequence stops at kSeqLen:
  // the words past it meet only coefficients at or above 19937, which are
  // zero, or outputs t >= 624, which are dropped).
  const PolyBuf pb = poly_buffer(poly);
  uint32_t i1 = c0;
  uint32_t n0 = poly_word(pb, c0 >> 5), n1 = poly_word(pb, (c0 >> 5) + 1), n2 = poly_word(pb, (c0 >> 5) + 2);
  while (i1 < c1) {
    extend<false>(ring, gen_hi, (int)i1 + kStepReach, lane);
    const uint32_t lim = (gen_hi >= kSeqLen) ? (uint32_t)kDeg : (uint32_t)(gen_hi - kStepReach);
    do {
      const uint32_t p0 = __builtin_amdgcn_readfirstlane(n0), p1 = __builtin_amdgcn_readfirstlane(n1),
                     p2 = __builtin_amdgcn_readfirstlane(n2);
      const uint32_t wn = (i1 + kStep) >> 5;
      n0 = poly_word(pb, wn);
      n1 = poly_word(pb, wn + 1);
      n2 = poly_word(pb, wn + 2);
      const uint32_t sh = i1 & 31;
      uint32_t b0 = (uint32_t)((((uint64_t)p1 << 32) | p0) >> sh);   // bits i1 .. i1 + 31
      uint32_t b1 = (uint32_t)((((uint64_t)p2 << 32) | p1) >> sh);   // bits i1 + 32 .. i1 + 63
      asm volatile("" : "+s"(b0), "+s"(b1));   // every test reads these two words
      group<0>(ring, i1, b0, b1, lane, acc, wa, wb, wc);
      group<kPer>(ring, i1 + kPer, b0, b1, lane, acc, wb, wc, wa);
      group<2 * kPer>(ring, i1 + 2 * kPer, b0, b1, lane, acc, wc, wa, wb);
      group<3 * kPer>(ring, i1 + 3 * kPer, b0, b1, lane, acc, wa, wb, wc);
      group<4 * kPer>(ring, i1 + 4 * kPer, b0, b1, lane, acc, wb, wc, wa);
      group<5 * kPer>(ring, i1 + 5 * kPer, b0, b1, lane, acc, wc, wa, wb);
      i1 += kStep;
    } while (i1 <= lim && i1 < c1);
  }
#pragma unroll
  for (int r = 0; r < kPer; r++) sum[r] = acc[r];
}

__device__ __forceinline__ void apply_poly(uint32_t* ring, const uint32_t* __restrict__ poly, int lane) {
  uint32_t acc[kPer];
  scan_range(ring, poly, lane, 0, (uint32_t)kDeg, acc);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kPer; r++) {
    const int t = kPer * lane + r;
    if (t < 624) ring[t] = (t == 0) ? (acc[r] & kUpper) : acc[r];
  }
  __syncthreads();
}

// apply_poly by kParts wavefronts of one workgroup, for few streams: the
// coefficients are cut into kParts ranges of kChunk (a multiple of kStep),
// wavefront w scans range w in its own ring rings[w] (first running the
// recurrence up to the range's start), and the partial sums, which add up to
// the whole because g(A) Y is linear in the coefficients, are XORed together
// through LDS and the result copied into every ring.  A lone stream's
// polynomial then takes the time of one range plus the recurrence up to it
// instead of the whole scan (the ranges' recurrence runs are repeated work,
// which is why many streams keep one wavefront each).
template <int kParts>
struct Split {
  static constexpr uint32_t kChunk = ((kDeg + kParts - 1) / kParts + kStep - 1) / kStep * kStep;
  static constexpr int kThreads = 64 * kParts;
  static constexpr int kWords = (624 + kThreads - 1) / kThreads;   // combined words per thread
  static_assert(kChunk * (kParts - 1) < (uint32_t)kDeg, "every range holds coefficients");
};

template <int kParts>
__device__ __forceinline__ void apply_poly_split(uint32_t (*rings)[kRing + kMirror], const uint32_t* __restrict__ poly,
                                                 int lane, int part) {
  using S = Split<kParts>;
  uint32_t* ring = rings[part];
  const uint32_t c0 = (uint32_t)part * S::kChunk;
  const uint32_t c1 = c0 + S::kChunk < (uint32_t)kDeg ? c0 + S::kChunk : (uint32_t)kDeg;
  uint32_t acc[kPer];
  scan_range(ring, poly, lane, c0, c1, acc);
  wave_lds_sync();   // the wavefront's reads of its ring are done
#pragma unroll
  for (int r = 0; r < kPer; r++) {
    const int t = kPer * lane + r;
    if (t < 624) ring[t] = acc[r];
  }
  __syncthreads();   // every partial in place
  uint32_t v[S::kWords];
#pragma unroll
  for (int k = 0; k < S::kWords; k++) {
    const int t = (int)threadIdx.x + S::kThreads * k;
    v[k] = 0;
    if (t < 624) {
#pragma unroll
      for (int p = 0; p < kParts; p++) v[k] ^= rings[p][t];
      if (t == 0) v[k] &= kUpper;
    }
  }
  __syncthreads();   // every partial read
#pragma unroll
  for (int k = 0; k < S::kWords; k++) {
    const int t = (int)threadIdx.x + S::kThreads * k;
    if (t < 624) {
#pragma unroll
      for (int p = 0; p < kParts; p++) rings[p][t] = v[k];
    }
  }
  __syncthreads();
}

// Lowest set bit of the multi-limb number N at or above bit `from`, or -1.
__device__ __forceinline__ int next_bit(const uint64_t (&N)[kMaxLimbs], int from) {
#pragma unroll
  for (int l = 0; l < kMaxLimbs; l++) {
    if (from < 64 * (l + 1)) {
      uint64_t w = N[l];
      if (from > 64 * l) w &= ~0ull << (from - 64 * l);
      if (w) return 64 * l + __builtin_ctzll(w);
    }
  }
  return -1;
}

// kParts = 1: one wavefront per stream; more: a workgroup of kParts
// wavefronts per stream, each polynomial applied by apply_poly_split.
template <int kParts>
__global__ void __launch_bounds__(64 * kParts) mt_jump_kernel(MtState* __restrict__ states, uint32_t count,
                                                     const uint64_t* __restrict__ dist, int nlimbs, int per_stream,
                                                     const uint64_t* __restrict__ ids, int block_e,
                                                     const MtState* __restrict__ base,
                                                     const MtState* __restrict__ top,
                                                     const uint32_t* __restrict__ ladder,
                                                     const uint32_t* __restrict__ diglo,
                                                     const uint32_t* __restrict__ dig8hi,
                                                     const uint32_t* __restrict__ blk, int blocks) {
  __shared__ __align__(16) uint32_t rings[kParts][kRing + kMirror];
  const uint32_t s = blockIdx.x;
  if (s >= count) return;
  // the scan is one long chain of dependent scalar tests and branches: where
  // its wavefronts share a SIMD with other kernels' (a served stream start
  // beside generation chunks), the highest wave priority lets the chain
  // issue first instead of waiting behind the others' VALU work
  __builtin_amdgcn_s_setprio(3);
  const int lane = threadIdx.x & 63;
  // the wavefront's part, uniform across it (its coefficient range is scanned
  // by scalar branching)
  const int part = kParts > 1 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : 0;
  uint32_t* ring = rings[part];
  // block splitting from the default state: start from the precomputed
  // state of the id's top 16 bits
  const bool digit_path = ids && block_e == kMtDigitE;
  const MtState* src = base ? base : states + s;
  if (digit_path && top) src = top + (ids[s] >> 48);
  uint64_t N[kMaxLimbs];
  for (int l = 0; l < kMaxLimbs; l++) N[l] = 0;
  if (ids) {
    const uint64_t id = ids[s];
    const int q = block_e >> 6, r = block_e & 63;
    N[q] = id << r;
    if (r && q + 1 < kMaxLimbs) N[q + 1] = id >> (64 - r);
  } else {
    const uint64_t* d = dist + (per_stream ? (size_t)s * nlimbs : 0);
    for (int l = 0; l < nlimbs; l++) N[l] = d[l];
  }
  for (int i = lane; i < 624; i += 64) ring[i] = src->mt[i];
  uint32_t idx = src->idx < 624u ? src->idx : 624u;
  wave_lds_sync();
  // the polynomials to apply, in order: for block splitting from a
  // block-aligned state, id * 2^432 with the low 48 bits of id as 16-bit
  // digits and the top 16 bits as two bytes, one table polynomial
  // x^(d 2^(432 + position)) per nonzero digit (the top bytes are already in
  // the start state when it came from the table of top-16-bit states);
  // otherwise one ladder polynomial x^(2^b) per set bit b of the distance
  // left after the rest of the current block.  One call site keeps a single
  // copy of the polynomial code.
  const bool use_digits = digit_path && idx == 624;
  const uint64_t id = ids ? ids[s] : 0;
  // distances D in whole sections: from a block boundary, and D within the
  // table, one whole-block polynomial per set bit of D (the state stays on a
  // boundary); otherwise the distance in outputs, D (624 2^kMtBlkFirst),
  // through the ladder
  const bool sec_units = blocks && !ids;
  const bool use_blocks = sec_units && idx == 624 && (N[0] >> kMtBlkPolys) == 0;
  if (sec_units && !use_blocks) {
    constexpr uint64_t kSec = 624ull << kMtBlkFirst;
    const uint64_t d = N[0];
    N[0] = d * kSec;
    N[1] = __umul64hi(d, kSec);
  }
  if (!use_digits && !use_blocks) {
    const uint64_t rest = 624 - idx;
    bool small = true;
    for (int l = 1; l < kMaxLimbs; l++) small = small && (N[l] == 0);
    small = small && (N[0] <= rest);
    if (small) {
      idx += (uint32_t)N[0];
      for (int l = 0; l < kMaxLimbs; l++) N[l] = 0;
    } else {
      uint64_t borrow = rest;
      for (int l = 0; l < kMaxLimbs && borrow; l++) {
        const uint64_t old = N[l];
        N[l] = old - borrow;
        borrow = old < borrow ? 1 : 0;
      }
      idx = 624;
    }
  }
  const int ndig = top ? kMtLoDigits : kMtLoDigits + 2;
  int pos = 0;
  for (;;) {
    const uint32_t* poly = nullptr;
    if (use_digits) {
      for (; pos < ndig && !poly; pos++) {
        if (pos < kMtLoDigits) {
          const uint32_t d = (uint32_t)(id >> (kMtLoBits * pos)) & (uint32_t)(kMtLoSize - 1);
          if (d) poly = diglo + ((size_t)pos * kMtLoSize + d) * 624;
        } else {
          const int j = pos - kMtLoDigits;
          const uint32_t d = (uint32_t)(id >> (48 + 8 * j)) & 255u;
          if (d) poly = dig8hi + ((size_t)j * 256 + d) * 624;
        }
      }
    } else {
      const int b = next_bit(N, pos);
      if (b >= 0) {
        poly = (use_blocks ? blk : ladder) + (size_t)b * 624;
        pos = b + 1;
      }
    }
    if (!poly) break;
    if constexpr (kParts > 1) apply_poly_split<kParts>(rings, poly, lane, part);
    else apply_poly(ring, poly, lane);
  }
  if (part) return;
  MtState* dst = states + s;
  for (int i = lane; i < 624; i += 64) dst->mt[i] = ring[i];
  if (lane == 0) {
    dst->idx = idx;
    dst->pad[0] = dst->pad[1] = dst->pad[2] = 0;
  }
}

// Start state of an MT19937 section tile of a batch: the task state moved
// D = first * kMtSection outputs on, a whole number of 624-word blocks, so
// the state keeps the task's block grid and its place in the block (idx)
// and equals the state sequential generation would reach.  x^D (one
// whole-block ladder polynomial per set bit of the section number) moves
// every word of the array D places along the sequence but leaves only the
// top bit of the oldest word exact; x^(-1) then steps the window one word
// back, so that the array's words 1..623 are the exact words 0..622 of the
// target window, and one step of the recurrence supplies its word 623.
// Section 0 is a copy.
__global__ void __launch_bounds__(64) mt_section_start_kernel(const BatchTile* __restrict__ tiles, uint32_t ntiles,
                                                              const BatchTask* __restrict__ tasks,
                                                              char* __restrict__ scratch,
                                                              const uint32_t* __restrict__ blk,
                                                              const uint32_t* __restrict__ inv) {
  __shared__ __align__(16) uint32_t ring[kRing + kMirror];
  const uint32_t t = blockIdx.x;
  if (t >= ntiles) return;
  const BatchTile tl = tiles[t];
  if (tl.kind != kTileMtSection) return;
  const int lane = threadIdx.x;
  const MtState* src = (const MtState*)tasks[tl.task].state_in;
  MtState* dst = (MtState*)(scratch + tl.starts);
  for (int i = lane; i < 624; i += 64) ring[i] = src->mt[i];
  const uint32_t idx = src->idx < 624u ? src->idx : 624u;
  __syncthreads();
  uint64_t sec = tl.first;
  if (sec == 0) {
    for (int i = lane; i < 624; i += 64) dst->mt[i] = ring[i];
  } else {
    for (int b = 0; sec; b++, sec >>= 1)
      if (sec & 1u) apply_poly(ring, blk + (size_t)b * 624, lane);
    apply_poly(ring, inv, lane);
    for (int i = lane; i < 623; i += 64) dst->mt[i] = ring[i + 1];
    if (lane == 0) dst->mt[623] = recur(ring[0], ring[1], ring[397]);
  }
  if (lane == 0) {
    dst->idx = idx;
    dst->pad[0] = dst->pad[1] = dst->pad[2] = 0;
  }
}

}  // namespace

hipError_t launch_batch_mt_starts(const DeviceTables& T, const BatchTile* tiles, uint32_t ntiles,
                                  const BatchTask* tasks, char* scratch, hipStream_t st) {
  if (!ntiles) return hipSuccess;
  hipLaunchKernelGGL(mt_section_start_kernel, dim3(ntiles), dim3(64), 0, st, tiles, ntiles, tasks, scratch, T.mtblk,
                     T.mtinv);
  return hipGetLastError();
}

hipError_t launch_mt_generate(MtState* states, uint32_t count, uint64_t n, int dtype, void* out, hipStream_t st) {
  switch (dtype) {
    case PRAND_U32: hipLaunchKernelGGL(mt_generate_kernel<PRAND_U32>, dim3(count), dim3(64), 0, st, states, count, n, out); break;
    case PRAND_F32: hipLaunchKernelGGL(mt_generate_kernel<PRAND_F32>, dim3(count), dim3(64), 0, st, states, count, n, out); break;
    default: hipLaunchKernelGGL(mt_generate_kernel<PRAND_F64>, dim3(count), dim3(64), 0, st, states, count, n, out); break;
  }
  return hipGetLastError();
}

hipError_t launch_mt_jump(const DeviceTables& T, MtState* states, uint32_t count, const JumpSpec& js,
                          const MtState* base, hipStream_t st) {
  // whole-section distances: one limb per stream
  if (js.mt_blocks && (js.ids || !js.per_stream || js.nlimbs != 1)) return hipErrorInvalidValue;
  if (count <= kMtSplit12MaxCount)
    hipLaunchKernelGGL(mt_jump_kernel<12>, dim3(count), dim3(64 * 12), 0, st, states, count, js.dist, js.nlimbs,
                       js.per_stream, js.ids, js.block_e, base, (const MtState*)js.mt_top, T.mt, T.mtdiglo, T.mtdig8hi,
                       T.mtblk, js.mt_blocks);
  else if (count <= kMtSplit8MaxCount)
    hipLaunchKernelGGL(mt_jump_kernel<8>, dim3(count), dim3(64 * 8), 0, st, states, count, js.dist, js.nlimbs,
                       js.per_stream, js.ids, js.block_e, base, (const MtState*)js.mt_top, T.mt, T.mtdiglo, T.mtdig8hi,
                       T.mtblk, js.mt_blocks);
  else
    hipLaunchKernelGGL(mt_jump_kernel<1>, dim3(count), dim3(64), 0, st, states, count, js.dist, js.nlimbs,
                       js.per_stream, js.ids, js.block_e, base, (const MtState*)js.mt_top, T.mt, T.mtdiglo, T.mtdig8hi,
                       T.mtblk, js.mt_blocks);
  return hipGetLastError();
}

}  // namespace prand
