// GM55, GQ58.3, GQ58.4 (v = 4, 3, 4; s = 8, 12, 8 elements): one lane per
// section of a stream (paper, equation rec1 with the Table 2 parameters).
//
// A lane steps all s elements of its section itself and packs their digits
// into words in registers (element 0 first, most significant bit first):
// v = 4 gives one word per step; GQ58.3 gives 36 bits per step, kept in a
// 64-bit bit buffer that yields 9 words per 8 steps.  No cross-lane work is
// needed per step.  The 64 runs of a wavefront lie in 64 different places, so
// words are written as in the register-state generators: chunks of CW words
// parked in LDS and stored transposed, 16-byte pieces of one chunk from
// consecutive lanes.
//
// Composite moduli: a section whose elements have not all collapsed (its
// start lies within n0 steps of a state that was not) runs exact mod-g steps
// first, four words at a time with plain stores, until every element of the
// wavefront has collapsed; then the mod-p recurrence takes over.
//
// The section's final state (when requested) is written at the step where it
// is reached: after len steps for v = 4; for GQ58.3 at the start of the last
// 8-step block the section touched, with the words of that block already
// used as the offset.
#pragma once

#include "dev_gm.h"
#include "regstream.h"

namespace prand {
namespace gm {

template <int G>
struct LaneShape {
  static constexpr int S = (G == 6) ? 12 : 8;
  static constexpr int V = (G == 6) ? 3 : 4;
};

struct ElemStart {
  uint64_t xc, xp;
  uint32_t off;
};

// One element of *in moved `start` outputs ahead, out of line: the jump code
// needs many registers and runs once per section.
template <int G>
__device__ __noinline__ ElemStart lane_start_elem(const GmState* in, int e, uint64_t start,
                                                  const uint64_t* __restrict__ ladder) {
  ElemStart r;
  r.off = load_at<G, true>(in, e, start, r.xc, r.xp, ladder);
  return r;
}

// Digits of one step of every element packed into the step's bits: v = 4
// returns the 32-bit word; GQ58.3 returns the 36-bit chunk right-aligned.
template <int G, bool kSlow>
__device__ __forceinline__ uint64_t lane_step(uint64_t (&sc)[LaneShape<G>::S], uint64_t (&sp)[LaneShape<G>::S],
                                              typename Eng<G>::F (&fc)[LaneShape<G>::S],
                                              typename Eng<G>::F (&fp)[LaneShape<G>::S]) {
  using E = Eng<G>;
  constexpr int S = LaneShape<G>::S;
  uint32_t d[S];
#pragma unroll
  for (int e = 0; e < S; e++) {
    if constexpr (kSlow) {
      const uint64_t nx = E::slow_step(sc[e], sp[e]);
      sp[e] = sc[e];
      sc[e] = nx;
      d[e] = E::slow_digit(nx);
    } else {
      const typename E::F nx = E::step(fc[e], fp[e]);
      fp[e] = fc[e];
      fc[e] = nx;
      d[e] = E::digit(nx);
    }
  }
  if constexpr (G == 6) {
    // element e at bits 33 - 3e .. 35 - 3e of the chunk
    const uint32_t hi = (d[0] << 1) | (d[1] >> 2);
    uint32_t lo = d[1] << 30;
#pragma unroll
    for (int e = 2; e < S; e++) lo |= d[e] << (33 - 3 * e);
    return ((uint64_t)hi << 32) | lo;
  } else {
    uint32_t w = d[0];
#pragma unroll
    for (int e = 1; e < S; e++) w = (w << 4) | d[e];
    return w;
  }
}

template <int G, int DT, int CW, bool kJump>
__device__ __forceinline__ void gmlane_wave(uint32_t* rows, bool live, const GmState* in, uint64_t start,
                                            uint64_t len, void* out, GmState* sout, bool coalesce,
                                            const uint64_t* __restrict__ ladder) {
  using E = Eng<G>;
  using F = typename E::F;
  constexpr int S = LaneShape<G>::S;
  constexpr int kPieces = CW / 4;                          // 16-byte pieces per chunk
  constexpr int per = (DT == PRAND_F64) ? CW / 2 : CW;      // values per chunk
  constexpr int es = (DT == PRAND_F64) ? 8 : 4;
  const int lane = threadIdx.x & 63;

  // exact start values
  uint64_t sc[S], sp[S];
  F fc[S], fp[S];   // set by to_fast() once every element has collapsed
  uint32_t off0 = 0;
#pragma unroll
  for (int e = 0; e < S; e++) sc[e] = sp[e] = 0;
  if (live) {
    if (kJump && start) {
#pragma unroll
      for (int e = 0; e < S; e++) {
        const ElemStart j = lane_start_elem<G>(in, e, start, ladder);
        sc[e] = j.xc;
        sp[e] = j.xp;
        off0 = j.off;
      }
    } else {
#pragma unroll
      for (int e = 0; e < S; e++) {
        sc[e] = in->xc[e];
        sp[e] = in->xp[e];
      }
      if (G == 6) off0 = in->off;
    }
  }
  // steps from the section's start state after which the final state is
  // written (none: ~0)
  const uint64_t total = off0 + len;
  const uint64_t save_at = (live && sout) ? (G == 6 ? 8 * (total / 9) : len) : ~0ull;
  const uint32_t off_end = (G == 6) ? (uint32_t)(total % 9) : 0u;
  uint64_t steps = 0;

  auto save = [&](bool fast) {
#pragma unroll
    for (int e = 0; e < S; e++) {
      sout->xc[e] = fast ? E::from_fast(fc[e]) : sc[e];
      sout->xp[e] = fast ? E::from_fast(fp[e]) : sp[e];
    }
#pragma unroll
    for (int e = S; e < 32; e++) {
      sout->xc[e] = 0;
      sout->xp[e] = 0;
    }
    sout->off = off_end;
    sout->pad = 0;
  };
  if (save_at == 0) save(false);

  // GQ58.3 bit buffer: nb valid bits at the top of buf
  uint64_t buf = 0;
  uint32_t nb = 0;
  auto word = [&](auto slow_tag) -> uint32_t {
    constexpr bool kSlow = decltype(slow_tag)::value;
    if constexpr (G == 6) {
      if (nb < 32) {
        const uint64_t cm = lane_step<G, kSlow>(sc, sp, fc, fp) << 28;   // chunk at the top
        if (++steps == save_at) save(!kSlow);
        const uint32_t w = (uint32_t)(buf >> 32) | (uint32_t)(cm >> (32 + nb));
        buf = cm << (32 - nb);
        nb += 4;
        return w;
      }
      const uint32_t w = (uint32_t)(buf >> 32);
      buf <<= 32;
      nb -= 32;
      return w;
    } else {
      const uint32_t w = (uint32_t)lane_step<G, kSlow>(sc, sp, fc, fp);
      if (++steps == save_at) save(!kSlow);
      return w;
    }
  };
  auto all_collapsed = [&]() {
    bool c = true;
#pragma unroll
    for (int e = 0; e < S; e++) c = c && E::collapsed(sc[e]) && E::collapsed(sp[e]);
    return c;
  };
  auto to_fast = [&]() {
#pragma unroll
    for (int e = 0; e < S; e++) {
      fc[e] = E::to_fast(sc[e]);
      fp[e] = E::to_fast(sp[e]);
    }
  };

  // words before the section's first output: the first off0 words of the
  // block (GQ58.3), dropped lane by lane
  uint64_t done = 0;   // outputs written so far (the same in every lane)
  if (__all(all_collapsed())) {
    to_fast();
    for (uint32_t k = 0; k < off0; k++) (void)word(std::false_type{});
  } else {
    for (uint32_t k = 0; k < off0; k++) (void)word(std::true_type{});
    // exact steps, four outputs at a time, until the wavefront has collapsed
    do {
#pragma unroll 1
      for (int q = 0; q < 4; q++) {
        const uint32_t w = word(std::true_type{});
        if (live && done + q < len) put<DT>(out, done + q, w);
      }
      done += 4;
    } while (!__all(all_collapsed()));
    to_fast();
  }

  // full chunks every live lane can still write (wavefront minimum)
  uint64_t my_rounds = live ? (len > done ? (len - done) / per : 0) : ~0ull;
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t other = __shfl_xor(my_rounds, o);
    my_rounds = other < my_rounds ? other : my_rounds;
  }
  const uint64_t rounds = (my_rounds == ~0ull || !coalesce) ? 0 : my_rounds;
  if (rounds) {
    char* const mine = live ? (char*)out + done * es : nullptr;
    char* dst[kPieces];
#pragma unroll
    for (int i = 0; i < kPieces; i++) {
      const int src = i * (64 / kPieces) + lane / kPieces;
      char* b = (char*)__shfl((unsigned long long)mine, src);
      dst[i] = b ? b + 16 * (lane % kPieces) : nullptr;
    }
    uint32_t* row = rows + lane * RegStage<CW>::kRowWords;
    for (uint64_t rd = 0; rd < rounds; rd++) {
      // one output per iteration: a single copy of the step code
#pragma unroll 1
      for (int q = 0; q < per; q++) {
        const uint32_t w = word(std::false_type{});
        if (DT == PRAND_F64) {
          const uint64_t u = __double_as_longlong((double)w * 0x1p-32);
          *(uint2*)(row + 2 * q) = make_uint2((uint32_t)u, (uint32_t)(u >> 32));
        } else if (DT == PRAND_F32) {
          row[q] = __float_as_uint((float)(w >> 8) * 0x1p-24f);
        } else {
          row[q] = w;
        }
      }
      wave_lds_sync();
      const uint64_t adv = rd * per * es;
#pragma unroll
      for (int i = 0; i < kPieces; i++) {
        const int src = i * (64 / kPieces) + lane / kPieces;
        const uint4 v = *(const uint4*)(rows + src * RegStage<CW>::kRowWords + 4 * (lane % kPieces));
        if (dst[i]) *(uint4*)(dst[i] + adv) = v;
      }
      wave_lds_sync();
    }
  }
  if (live) {
    for (uint64_t i = done + rounds * per; i < len; i++) put<DT>(out, i, word(std::false_type{}));
  }
}

}  // namespace gm
}  // namespace prand
