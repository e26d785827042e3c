// MT19937 device code shared by the MT19937 kernels and the batched kernel.
#pragma once

#include "prand_impl.h"

namespace prand {
namespace mt {

constexpr uint32_t kUpper = 0x80000000u;
constexpr uint32_t kLower = 0x7FFFFFFFu;
constexpr uint32_t kMatA = 0x9908B0DFu;

// y ^ ((y << k) & mask) as one three-input op (gfx950 v_bitop3_b32; truth
// table 0x78 = src0 ^ (src1 & src2))
__device__ __forceinline__ uint32_t xor_and(uint32_t a, uint32_t b, uint32_t m) {
  return __builtin_amdgcn_bitop3_b32(a, b, m, 0x78);
}
__device__ __forceinline__ uint32_t temper(uint32_t y) {
  y ^= y >> 11;
  y = xor_and(y, y << 7, 0x9D2C5680u);
  y = xor_and(y, y << 15, 0xEFC60000u);
  return y ^ (y >> 18);
}
// x_{j+624} from x_j (upper bit), x_{j+1} (lower bits), x_{j+397}
__device__ __forceinline__ uint32_t recur(uint32_t xj, uint32_t xj1, uint32_t xjm) {
  const uint32_t y = (xj & kUpper) | (xj1 & kLower);
  return xjm ^ (y >> 1) ^ ((xj1 & 1u) ? kMatA : 0u);
}

template <int DT>
__device__ __forceinline__ void put(void* out, uint64_t i, uint32_t w) {
  if (DT == PRAND_U32) ((uint32_t*)out)[i] = w;
  else if (DT == PRAND_F32) ((float*)out)[i] = (float)(w >> 8) * 0x1p-24f;
  else ((double*)out)[i] = (double)w * 0x1p-32;
}

// A piece of a twist phase: words j = j0 + lane + 64 k (k < K, j < j1)
// become recur(mt[j], mt[j + 1], mt[j + off]) (word 623's successor is word
// 0).  Every word a phase reads is either untouched by it or renewed by an
// earlier phase, so a piece issues all its loads before any of its stores:
// one LDS latency per K slices of 64 words instead of one per slice (a lone
// wavefront, as in batched and served MT19937 tasks, is bound by that
// latency).  kOut: renewed words below `want` are also tempered and stored
// at out[pos + j] straight from registers.
template <int DT, int K, bool kOut = true>
__device__ __forceinline__ void twist_phase(uint32_t* mt, int j0, int j1, int off, int want, uint64_t pos, void* out) {
  const int lane = threadIdx.x & 63;
  uint32_t a[K], b[K], c[K];
#pragma unroll
  for (int k = 0; k < K; k++) {
    const int j = j0 + lane + 64 * k;
    if (j < j1) {
      a[k] = mt[j];
      b[k] = mt[j == 623 ? 0 : j + 1];
      c[k] = mt[j + off];
    }
  }
  // lane 63's mt[j + 1] is lane 0's word of the next slice (maybe in the
  // next piece): no store may be scheduled above these loads (one
  // wavefront's LDS operations then run in issue order)
  asm volatile("" ::: "memory");
#pragma unroll
  for (int k = 0; k < K; k++) {
    const int j = j0 + lane + 64 * k;
    if (j < j1) {
      const uint32_t v = recur(a[k], b[k], c[k]);
      mt[j] = v;
      if (kOut && j < want) put<DT>(out, pos + j, temper(v));
    }
  }
}

// A twist phase out of place: words j = j0 + lane + 64 k (k < K, j < j1) of
// the new block N from the old block O.  Phase one (kFirst) reads O[j + 397];
// the later phases read N[j - 227], renewed by an earlier phase; word 623
// pairs with N[0].  Nothing the phase reads is written by it.
template <int K, bool kFirst>
__device__ __forceinline__ void twist_phase_oop(const uint32_t* O, uint32_t* N, int j0, int j1) {
  const int lane = threadIdx.x & 63;
  uint32_t a[K], b[K], c[K];
#pragma unroll
  for (int k = 0; k < K; k++) {
    const int j = j0 + lane + 64 * k;
    if (j < j1) {
      a[k] = O[j];
      b[k] = j == 623 ? N[0] : O[j + 1];
      c[k] = kFirst ? O[j + 397] : N[j - 227];
    }
  }
#pragma unroll
  for (int k = 0; k < K; k++) {
    const int j = j0 + lane + 64 * k;
    if (j < j1) N[j] = recur(a[k], b[k], c[k]);
  }
}

// the block after O, written to N (three out-of-place phases)
__device__ __forceinline__ void twist_oop(const uint32_t* O, uint32_t* N) {
  twist_phase_oop<4, true>(O, N, 0, 227);
  wave_lds_sync();
  twist_phase_oop<4, false>(O, N, 227, 454);
  wave_lds_sync();
  twist_phase_oop<3, false>(O, N, 454, 624);
  wave_lds_sync();
}

template <int DT>
__device__ __forceinline__ void put4(char* out, int q, uint4 w) {
  const uint32_t t0 = temper(w.x), t1 = temper(w.y), t2 = temper(w.z), t3 = temper(w.w);
  if (DT == PRAND_U32) {
    store_out16<DT>(out + 16 * q, make_uint4(t0, t1, t2, t3));
  } else if (DT == PRAND_F32) {
    store_out16<DT>(out + 16 * q, make_uint4(__float_as_uint((float)(t0 >> 8) * 0x1p-24f),
                                         __float_as_uint((float)(t1 >> 8) * 0x1p-24f),
                                         __float_as_uint((float)(t2 >> 8) * 0x1p-24f),
                                         __float_as_uint((float)(t3 >> 8) * 0x1p-24f)));
  } else {
    const uint64_t d0 = __double_as_longlong((double)t0 * 0x1p-32), d1 = __double_as_longlong((double)t1 * 0x1p-32);
    const uint64_t d2 = __double_as_longlong((double)t2 * 0x1p-32), d3 = __double_as_longlong((double)t3 * 0x1p-32);
    store_out16<DT>(out + 32 * q, make_uint4((uint32_t)d0, (uint32_t)(d0 >> 32), (uint32_t)d1, (uint32_t)(d1 >> 32)));
    store_out16<DT>(out + 32 * q + 16, make_uint4((uint32_t)d2, (uint32_t)(d2 >> 32), (uint32_t)d3, (uint32_t)(d3 >> 32)));
  }
}

// Two consecutive blocks A then B written out as 16-byte pieces (312 pieces
// of four words, five per lane): 1248 words, 39 whole 128-byte lines when
// `out` is line-aligned.  out 16-byte aligned; A, B 16-byte aligned LDS.
template <int DT>
__device__ __forceinline__ void write_pair(const uint32_t* A, const uint32_t* B, char* out) {
  const int lane = threadIdx.x & 63;
  uint4 w[5];
#pragma unroll
  for (int r = 0; r < 5; r++) {
    const int q = lane + 64 * r;
    if (q < 312) w[r] = q < 156 ? *(const uint4*)(A + 4 * q) : *(const uint4*)(B + 4 * (q - 156));
  }
#pragma unroll
  for (int r = 0; r < 5; r++) {
    const int q = lane + 64 * r;
    if (q < 312) put4<DT>(out, q, w[r]);
  }
}

// A whole renewed block written out as 16-byte pieces: lane l tempers the
// words 4q .. 4q + 3 for q = l, l + 64, l + 128 (q < 156) and stores them at
// out + 16 q (u32/f32) or out + 32 q (f64, two pieces).  `out` is 16-byte
// aligned; mt is 16-byte aligned LDS.
template <int DT>
__device__ __forceinline__ void write_block(const uint32_t* mt, char* out) {
  const int lane = threadIdx.x & 63;
  uint4 w[3];
#pragma unroll
  for (int r = 0; r < 3; r++) {
    const int q = lane + 64 * r;
    if (q < 156) w[r] = *(const uint4*)(mt + 4 * q);
  }
#pragma unroll
  for (int r = 0; r < 3; r++) {
    const int q = lane + 64 * r;
    if (q < 156) put4<DT>(out, q, w[r]);
  }
}

// One wavefront generates n outputs of one stream: state *in (copied into
// the LDS block mt[624], 16-byte aligned), outputs at out, advanced state to
// *sout (may be the same object as *in).  A twist renews the block in three
// dependency phases (words 0..226 read old words 397..623; 227..453 read
// words renewed in phase one; 454..623 read phase two and word 0), each
// parallel across the lanes.  A whole block whose outputs start 16-byte
// aligned is twisted first (one piece per phase) and then tempered and
// written out from LDS as 16-byte pieces (one vector store per four words
// instead of four); a partial block tempers and stores renewed words
// straight from registers.  kPairs (mt then holds 1248 words): while two
// whole blocks remain, the first is twisted from mt into mt + 624 and the
// second back into mt, and the two are written out together (1248 words:
// whole 128-byte lines, where a single block ends in the middle of one;
// measured about 5 % faster for 65536 streams).  The LDS block is private to
// the wavefront (wavefront-level ordering only).
template <int DT, bool kPairs = false>
__device__ __forceinline__ void gen_wave(uint32_t* mt, const MtState* in, MtState* sout, uint64_t n, void* out) {
  constexpr int es = (DT == PRAND_F64) ? 8 : 4;
  const int lane = threadIdx.x & 63;
  for (int i = lane; i < 624; i += 64) mt[i] = in->mt[i];
  uint32_t idx = in->idx < 624u ? in->idx : 624u;   // an index past the block means "block used up"
  wave_lds_sync();
  // rest of the current block
  const uint64_t first = (uint64_t)(624 - idx) < n ? (uint64_t)(624 - idx) : n;
  for (uint32_t i = lane; i < first; i += 64) put<DT>(out, i, temper(mt[idx + i]));
  uint64_t pos = first;
  idx += (uint32_t)first;
  // every later block starts 624 * es bytes (a multiple of 16) further on
  const bool vec = (((uintptr_t)out + pos * es) & 15) == 0;
  while (pos < n) {
    const uint64_t left = n - pos;
    if (kPairs && vec && left >= 1248) {
      twist_oop(mt, mt + 624);
      twist_oop(mt + 624, mt);
      write_pair<DT>(mt + 624, mt, (char*)out + pos * es);
      wave_lds_sync();
      pos += 1248;
      idx = 624;
      continue;
    }
    const int want = left < 624 ? (int)left : 624;
    if (vec && want == 624) {
      twist_phase<DT, 4, false>(mt, 0, 227, 397, 0, 0, nullptr);
      wave_lds_sync();
      twist_phase<DT, 4, false>(mt, 227, 454, -227, 0, 0, nullptr);
      wave_lds_sync();
      twist_phase<DT, 3, false>(mt, 454, 624, -227, 0, 0, nullptr);
      wave_lds_sync();
      write_block<DT>(mt, (char*)out + pos * es);
    } else {
      // phases in pieces of two 64-word slices: the loads of four slices at
      // once measured the same for a lone wavefront but took 60 instead of 56
      // VGPRs in the batch kernel that shares this code with the v = 1 GM/GQ
      // tiles, which upset the balance of the batch's concurrent kernels
      twist_phase<DT, 2>(mt, 0, 128, 397, want, pos, out);
      twist_phase<DT, 2>(mt, 128, 227, 397, want, pos, out);
      wave_lds_sync();
      twist_phase<DT, 2>(mt, 227, 355, -227, want, pos, out);
      twist_phase<DT, 2>(mt, 355, 454, -227, want, pos, out);
      wave_lds_sync();
      twist_phase<DT, 2>(mt, 454, 582, -227, want, pos, out);
      twist_phase<DT, 1>(mt, 582, 624, -227, want, pos, out);
    }
    wave_lds_sync();
    pos += want;
    idx = want;
  }
  for (int i = lane; i < 624; i += 64) sout->mt[i] = mt[i];
  if (lane == 0) {
    sout->idx = idx;
    sout->pad[0] = sout->pad[1] = sout->pad[2] = 0;
  }
}

}  // namespace mt
}  // namespace prand
