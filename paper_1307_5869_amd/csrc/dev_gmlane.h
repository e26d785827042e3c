// GM55, GQ58.3, GQ58.4 (v = 4, 3, 4; s = 8, 12, 8 elements): one lane per
// section of a stream (paper, equation rec1 with the Table 2 parameters).
//
// A lane steps all s elements of its section itself and packs their digits
// in registers (element 0 first, most significant bit first): v = 4 gives
// one word per step; GQ58.3 gives 36 bits per step, which a bit buffer turns
// into 9 words per 8 steps.  No cross-lane work is needed per step.  Steps
// run in pairs over two value arrays used in turn (a step writes the new
// value over the one two steps back), so no value is ever copied.
//
// Outputs are counted in a frame that starts at the block boundary where the
// section's state sits: a GQ58.3 state consumed `off` words of its block, so
// the section's outputs are frame outputs off .. off + len - 1.  Every lane
// of a wavefront steps in lockstep from such a boundary, so all lanes make
// the same number of outputs per step.  Outputs go to a per-lane ring in LDS;
// every F words (16 in the many-stream kernel) the wavefront stores them
// transposed: in each store instruction F / 4 consecutive lanes write the
// 16-byte pieces of one lane's 4F-byte run (whole pieces that lie inside the
// section and are 16-byte aligned; the others word by word).
//
// Composite moduli: a wavefront with an element that has not collapsed (a
// section within n0 steps of a state that had not) first runs exact mod-g
// steps with plain stores, until every element of the wavefront has
// collapsed; then the mod-p recurrence takes over.  A section that starts by
// a jump (always past n0 steps) starts collapsed.
//
// The section's final state (when requested) is written at the step where it
// is reached: after len steps for v = 4; for GQ58.3 at the start of the last
// 8-step block the section touched, with the words of that block already
// used as the offset.
#pragma once

#include "dev_gm.h"

namespace prand {
namespace gm {

template <int G>
struct LaneShape {
  static constexpr int S = (G == 6) ? 12 : 8;
};

// LDS per wavefront: a ring of 2F words per lane in rows of 2F + 4 words
// (16-byte aligned; the exact steps of a composite start use up to 18 words
// of the row), flushed F words at a time (F = 32: a 48-word ring).  The
// many-stream kernels use F = 16 (64-byte runs per lane, 9 KB per
// wavefront: with 4-wavefront workgroups 4 per CU), F = 32 for GQ58.3
// (whole 128-byte lines, 13 KB); the batched kernels, which share the CUs
// with the other classes, F = 8 (32-byte runs, 5 KB per wavefront).
template <int F>
struct LaneRing {
  static constexpr int kFlush = F;
  static constexpr int kRing = (F == 32) ? 48 : 2 * F;   // holds F + 5 words between flushes
  static constexpr int kRow = kRing + 4;
  static constexpr int kWaveWords = 64 * kRow;
  __device__ static uint32_t slot(uint32_t w) { return (kRing & (kRing - 1)) ? w % kRing : w & (kRing - 1); }
};
constexpr int kLaneFlushWide = 16;
constexpr int kLaneFlushNarrow = 8;

template <int G>
struct FastPair {
  typename Eng<G>::F yc, yp;
};

// m0 a + m1 b mod p for the prime part of GM55 / GQ58 (all operands < p)
template <int G>
__device__ __forceinline__ uint64_t lane_mulsum(uint64_t m0, uint64_t a, uint64_t m1, uint64_t b) {
  if constexpr (G == 3) {
    return fold_special<G>((u128)m0 * a + (u128)m1 * b, 51, 129, Eng<3>::p);
  } else {
    // p = 2^29 - 3: products below 2^58, folded twice with 2^29 = 3 (mod p)
    const uint64_t t = m0 * a + m1 * b;                                           // < 2^59
    const uint64_t u = (t & 0x1FFFFFFFull) + 3ull * (t >> 29);                    // < 2^32 + 2^29
    const uint32_t w = (uint32_t)(u & 0x1FFFFFFFull) + 3u * (uint32_t)(u >> 29);  // < 2^29 + 24
    return w >= EngGQ<1>::kP ? w - EngGQ<1>::kP : w;
  }
}

// Element e of *in moved nsteps >= n0 ensemble steps ahead, in the fast
// (collapsed, mod p) representation: exact steps until the element has
// collapsed, then one ladder matrix M^(2^b) mod p per set bit b of the rest.
template <int G>
__device__ __forceinline__ FastPair<G> lane_jump_fast(const GmState* in, int e, uint64_t nsteps,
                                                   const uint64_t* __restrict__ ladder) {
  using E = Eng<G>;
  uint64_t xc = in->xc[e], xp = in->xp[e];
  if (!(E::collapsed(xc) && E::collapsed(xp))) {
    const int n0 = kGmParams[G].n0;
    for (int i = 0; i < n0; i++) {
      const uint64_t nx = E::slow_step(xc, xp);
      xp = xc;
      xc = nx;
    }
    nsteps -= n0;
  }
  uint64_t yc = xc >> E::t, yp = xp >> E::t;
  const uint64_t* L = ladder + (size_t)G * kLadder * 4;
  while (nsteps) {
    const int b = __builtin_ctzll(nsteps);
    nsteps &= nsteps - 1;
    const uint64_t* M = L + (size_t)b * 4;
    const uint64_t nc = lane_mulsum<G>(M[0], yc, M[1], yp);
    const uint64_t np = lane_mulsum<G>(M[2], yc, M[3], yp);
    yc = nc;
    yp = np;
  }
  FastPair<G> r;   // the ladder gives exact residues; the kernels' form may be offset
  r.yc = E::to_fast(yc << E::t);
  r.yp = E::to_fast(yp << E::t);
  return r;
}

// One step of every element: nw[e] = step(cur[e], nw[e]) (nw holds the
// values one step back and receives the new ones); the digits packed into
// the step's bits: v = 4 returns the 32-bit word, GQ58.3 the 36-bit chunk
// right-aligned.
template <int G, bool kSlow, class T>
__device__ __forceinline__ uint64_t lane_step(const T (&cur)[LaneShape<G>::S], T (&nw)[LaneShape<G>::S]) {
  using E = Eng<G>;
  constexpr int S = LaneShape<G>::S;
  uint32_t d[S];
#pragma unroll
  for (int e = 0; e < S; e++) {
    if constexpr (kSlow) {
      nw[e] = E::slow_step(cur[e], nw[e]);
      d[e] = E::slow_digit(nw[e]);
    } else {
      nw[e] = E::step(cur[e], nw[e]);
      d[e] = E::digit(nw[e]);
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

// Store ring words [flushed, flushed + nw) of every lane of the wavefront
// (nw <= F, flushed a multiple of F): in store instruction i, the P = F / 4
// lanes P j .. P j + P - 1 write the 16-byte pieces of lane (64 / P) i + j's
// run.  mine: the
// lane's section output (null for a dead lane); the ring starts at frame
// output f0; the section holds frame outputs [off0, total).  (Kernels here
// make no calls: a call would keep every value live across it in extra
// registers.)
template <int DT, int F>
__device__ __forceinline__ void lane_flush(const uint32_t* rows, uint32_t flushed, uint32_t nw, uint64_t f0, char* mine,
                                        uint64_t off0, uint64_t total) {
  constexpr int kw = (DT == PRAND_F64) ? 2 : 1;
  constexpr int es = 4 * kw;
  const int lane = threadIdx.x & 63;
  wave_lds_sync();
  constexpr int P = F / 4;   // 16-byte pieces per run
#pragma unroll
  for (int i = 0; i < P; i++) {
    const int src = i * (64 / P) + lane / P;
    const uint32_t pw = flushed + 4 * (lane % P);   // first ring word of the piece
    char* const o = (char*)__shfl((unsigned long long)mine, src);
    const uint64_t so = __shfl(off0, src), st = __shfl(total, src);
    const uint32_t* r = rows + src * LaneRing<F>::kRow + LaneRing<F>::slot(pw);
    if (o && pw < flushed + nw) {
      const uint64_t fo = f0 + pw / kw;   // frame output of the piece's first word
      char* const d = o + (fo - so) * es;
      if (flushed + nw - pw >= 4 && fo >= so && fo + 4 / kw <= st && (uintptr_t)d % 16 == 0) {
        *(uint4*)d = *(const uint4*)r;
      } else {
        for (int t = 0; t < 4 && pw + t < flushed + nw; t += kw) {
          const uint64_t g = f0 + (pw + t) / kw;
          if (g >= so && g < st) {
            if (kw == 2) *(uint2*)(o + (g - so) * es) = *(const uint2*)(r + t);
            else *(uint32_t*)(o + (g - so) * es) = r[t];
          }
        }
      }
    }
  }
  wave_lds_sync();
}

template <int G, int DT, bool kJump, int FW = kLaneFlushWide>
__device__ __forceinline__ void gmlane_wave(uint32_t* rows, bool live, const GmState* in, uint64_t start,
                                            uint64_t len, void* out, GmState* sout,
                                            const uint64_t* __restrict__ ladder) {
  using E = Eng<G>;
  using F = typename E::F;
  constexpr int S = LaneShape<G>::S;
  constexpr int kw = (DT == PRAND_F64) ? 2 : 1;   // ring words per output
  const int lane = threadIdx.x & 63;
  uint32_t* row = rows + lane * LaneRing<FW>::kRow;

  // start values: jumped sections in the fast representation; the others
  // exact in *in (converted below)
  F fa[S], fb[S];   // fa current after an even number of steps
  uint32_t off0 = 0;
  uint64_t nsteps = 0;
  bool jumped = false;
  if (live && kJump && start) {
    nsteps = start;
    if (G == 6) {   // words from the block start -> whole blocks of 8 steps
      const uint64_t w = (uint64_t)in->off + start;
      nsteps = 8 * (w / 9);
      off0 = (uint32_t)(w % 9);
    }
#pragma unroll
    for (int e = 0; e < S; e++) {
      const FastPair<G> j = lane_jump_fast<G>(in, e, nsteps, ladder);
      fa[e] = j.yc;
      fb[e] = j.yp;
    }
    jumped = true;
  } else if (G == 6 && live) {
    off0 = in->off;
  }
  const uint64_t total = live ? off0 + len : 0;   // frame outputs this lane needs
  // steps after which the final state is written (none: ~0)
  const uint64_t save_at = (live && sout) ? (G == 6 ? 8 * (total / 9) : len) : ~0ull;
  const uint32_t off_end = (G == 6) ? (uint32_t)(total % 9) : 0u;

  // steps the wavefront runs: enough for every lane's outputs (GQ58.3:
  // 8 steps per 9 words) and its final state, rounded up to a pair
  uint64_t need = (G == 6) ? (total * 8 + 8) / 9 : total;
  if (save_at != ~0ull && save_at > need) need = save_at;
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t other = __shfl_xor(need, o);
    need = other > need ? other : need;
  }
  const uint64_t pairs = (need + 1) / 2;

  // sout may be another section's input (the sections of a stream share
  // it): every slot is written only after every lane has read that slot
  // (element e's exact steps read element e before writing it; the fast
  // steps come after all reads).
  auto save_tail = [&]() {   // the blob's unused slots, offset, pad
#pragma unroll
    for (int e = S; e < 32; e++) {
      sout->xc[e] = 0;
      sout->xp[e] = 0;
    }
    sout->off = off_end;
    sout->pad = 0;
  };
  // (the volatile asm keeps the conversion to exact values inside the rare
  // save branch instead of letting it run ahead on every step)
  auto save_fast = [&](const F (&cur)[S], const F (&prev)[S]) {
#pragma unroll
    for (int e = 0; e < S; e++) {
      F c = cur[e], q = prev[e];
      asm volatile("" : "+v"(c), "+v"(q));
      sout->xc[e] = E::from_fast(c);
      sout->xp[e] = E::from_fast(q);
    }
    save_tail();
  };
  // frame outputs made so far (the same in every lane), GQ58.3 bit buffer
  uint64_t f = 0;
  uint64_t steps = 0;
  uint64_t buf = 0;
  uint32_t nb = 0;
  auto put_frame = [&](uint32_t w) {   // plain store of frame output f
    if (live && f >= off0 && f < total) put<DT>(out, f - off0, w);
    f++;
  };

  // Composite moduli: unless every element of the wavefront has collapsed,
  // every lane first runs K = n0 (rounded up to a pair) exact steps, element
  // by element, OR-ing the digits into its LDS row (K words for v = 4, the
  // 18-word bit stream of 16 steps for GQ58.3); every element has collapsed
  // after them.
  constexpr int K = (kGmParams[G].n0 + 1) & ~1;
  constexpr int KW = (G == 6) ? (K * 36 + 31) / 32 : K;   // words the K steps make
  static_assert(G != 6 || K == 16, "GQ58.3: 16 exact steps make whole words");
  static_assert(KW <= LaneRing<FW>::kRow, "exact steps fit the LDS row");
  bool coll = true;
  if (!jumped && live) {
#pragma unroll
    for (int e = 0; e < S; e++) coll = coll && E::collapsed(in->xc[e]) && E::collapsed(in->xp[e]);
  }
  uint64_t p = 0;   // pairs done
  if (!__all(coll)) {
#pragma unroll
    for (int w = 0; w < KW; w++) row[w] = 0;
#pragma unroll
    for (int e = 0; e < S; e++) {
      uint64_t xc = jumped ? E::from_fast(fa[e]) : (live ? in->xc[e] : 0);
      uint64_t xp = jumped ? E::from_fast(fb[e]) : (live ? in->xp[e] : 0);
#pragma unroll 1
      for (int u = 0; u < K; u++) {
        const uint64_t nx = E::slow_step(xc, xp);
        xp = xc;
        xc = nx;
        const uint32_t d = E::slow_digit(nx);
        if constexpr (G == 6) {
          const int B = 36 * u + 3 * e;   // stream bit of the digit's top bit
          const int w = B >> 5, b = B & 31;
          if (b <= 29) {
            row[w] |= d << (29 - b);
          } else {
            row[w] |= d >> (b - 29);
            row[w + 1] |= d << (61 - b);
          }
        } else {
          row[u] |= d << (28 - 4 * e);
        }
        if ((uint64_t)(u + 1) == save_at) {
          sout->xc[e] = xc;
          sout->xp[e] = xp;
        }
      }
      fa[e] = E::to_fast(xc);
      fb[e] = E::to_fast(xp);
    }
    if (save_at >= 1 && save_at <= (uint64_t)K) save_tail();
    for (int w = 0; w < KW; w++) put_frame(row[w]);
    steps = K;
    p = K / 2;
  } else if (!jumped) {
#pragma unroll
    for (int e = 0; e < S; e++) {
      fa[e] = live ? E::to_fast(in->xc[e]) : 0;
      fb[e] = live ? E::to_fast(in->xp[e]) : 0;
    }
  }

  // one step's bits -> outputs (v = 4: one; GQ58.3: one or two), each
  // handed to emit(word)
  auto outputs = [&](uint64_t bits, auto&& emit) {
    if constexpr (G == 6) {
      const uint64_t cm = bits << 28;   // chunk at the top
      emit((uint32_t)(buf >> 32) | (uint32_t)(cm >> (32 + nb)));
      buf = cm << (32 - nb);
      nb += 4;
      if (nb >= 32) {
        emit((uint32_t)(buf >> 32));
        buf <<= 32;
        nb -= 32;
      }
    } else {
      emit((uint32_t)bits);
    }
  };

  // fast steps; outputs through the LDS ring
  const uint64_t f0 = f;   // frame output of ring word 0
  uint32_t appended = 0, flushed = 0;   // ring words (ring index = counter % 32)
  char* const mine = live ? (char*)out : nullptr;
  auto put_ring = [&](uint32_t w) {
    const uint32_t at = LaneRing<FW>::slot(appended);
    if (DT == PRAND_F64) {
      const uint64_t u = __double_as_longlong((double)w * 0x1p-32);
      *(uint2*)(row + at) = make_uint2((uint32_t)u, (uint32_t)(u >> 32));
    } else if (DT == PRAND_F32) {
      row[at] = __float_as_uint((float)(w >> 8) * 0x1p-24f);
    } else {
      row[at] = w;
    }
    appended += kw;
    f++;
  };
  // at most 6 ring words per pair: a flush after every pair keeps at most
  // FW + 5 words in the ring
  for (; p < pairs; p++) {
    outputs(lane_step<G, false>(fa, fb), put_ring);
    if (++steps == save_at) save_fast(fb, fa);
    outputs(lane_step<G, false>(fb, fa), put_ring);
    if (++steps == save_at) save_fast(fa, fb);
    if (appended - flushed >= (uint32_t)FW) {
      lane_flush<DT, FW>(rows, flushed, FW, f0, mine, off0, total);
      flushed += FW;
    }
  }
  if (appended != flushed) lane_flush<DT, FW>(rows, flushed, appended - flushed, f0, mine, off0, total);
  // a final state reached at step 0 (a GQ58.3 section within its first
  // block, or an empty one) is the start state; it is written last, since
  // sout may be another section's input: start values again from *in
  if (save_at == 0) {
#pragma unroll 1
    for (int e = 0; e < S; e++) {
      uint64_t xc = in->xc[e], xp = in->xp[e];
      if (jumped) {
        const FastPair<G> j = lane_jump_fast<G>(in, e, nsteps, ladder);
        xc = E::from_fast(j.yc);
        xp = E::from_fast(j.yp);
      }
      sout->xc[e] = xc;
      sout->xp[e] = xp;
    }
    save_tail();
  }
}

}  // namespace gm
}  // namespace prand
