// Generation for generators whose whole state fits in a lane's registers
// (MRG32K3A, LFSR113): one lane per section of a stream.
//
// A section starts from a state jumped to its first output and fills a
// contiguous run of the output.  The 64 runs of a wavefront lie in 64
// different places, so each lane produces its outputs in chunks of CW words
// (CW = 32: 128 bytes, 32 u32/f32 or 16 f64 values), parks them in LDS, and
// the wavefront stores them transposed: in each store instruction the CW/4
// consecutive lanes of a group write the 16-byte pieces of one chunk (CW = 32:
// eight whole 128-byte lines per instruction).  Rounds run while any lane
// still has a full chunk to write (a lane whose run is shorter sits out the
// later rounds); the rest of each run, fewer than one chunk, is stored lane
// by lane.
//
// regstream_wave() is the wavefront routine shared by the many-stream kernel
// below and by the batched generation kernel.
#pragma once

#include <cstdlib>

#include "prand_impl.h"

namespace prand {

template <int CW>
struct RegStage {
  static constexpr int kRowWords = CW + 4;            // padded row, 16-byte aligned
  static constexpr int kWaveWords = 64 * kRowWords;   // LDS words per wavefront
};

template <int DT>
__device__ __forceinline__ void put_word(void* out, uint64_t i, uint32_t w, double f64v) {
  if (DT == PRAND_U32) ((uint32_t*)out)[i] = w;
  else if (DT == PRAND_F32) ((float*)out)[i] = (float)(w >> 8) * 0x1p-24f;
  else ((double*)out)[i] = f64v;
}

// One lane's section: live lanes start from *in (jumped `start` outputs
// ahead: by the jump matrix sec_mat when it is given, else through the
// ladder), write `len` values at `out` (element pointer of the run) and, when
// `sout` is set, store the advanced state there.  `coalesce`: every run start
// is 16-byte aligned (transposed stores allowed).  All 64 lanes must call.
// kJump = false: the caller guarantees start == 0 (no jump code is built).
//
// G: State, Regs, static load(State) -> Regs, static save(Regs) -> State,
// static jump(State&, uint64_t distance, const uint32_t* ladder),
// static apply(State&, const uint32_t* jump matrix),
// static next(Regs&) -> uint32_t word, static f64(uint32_t) -> double.
template <class G, int DT, int CW, bool kJump = true>
__device__ __forceinline__ void regstream_wave(uint32_t* rows, bool live, const typename G::State* in, uint64_t start,
                                               uint64_t len, void* out, typename G::State* sout, bool coalesce,
                                               const uint32_t* __restrict__ ladder,
                                               const uint32_t* __restrict__ sec_mat = nullptr) {
  constexpr int kPieces = CW / 4;                            // 16-byte pieces per chunk
  constexpr int per = (DT == PRAND_F64) ? CW / 2 : CW;        // values per chunk
  constexpr int es = (DT == PRAND_F64) ? 8 : 4;
  const int lane = threadIdx.x & 63;
  typename G::State st = {};
  if (live) {
    st = *in;
    if (kJump && sec_mat) G::apply(st, sec_mat);
    else if (kJump && start) G::jump(st, start, ladder);
  }
  typename G::Regs r = G::load(st);
  // full chunks of this lane, and the most any lane of the wavefront has:
  // round rd stores the chunks of the lanes with rd < their own count, so
  // lanes of uneven lengths (the short last section of a task) keep the
  // transposed stores for all their full chunks
  const uint64_t my_rounds = (live && coalesce) ? len / per : 0;
  uint64_t rounds = my_rounds;
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t other = __shfl_xor(rounds, o);
    rounds = other > rounds ? other : rounds;
  }
  if (rounds) {
    // destination of piece (lane % kPieces) of each source lane's chunk, one
    // per store instruction, and that source lane's chunk count
    char* const mine = live ? (char*)out : nullptr;
    char* dst[kPieces];
    uint64_t src_rounds[kPieces];
#pragma unroll
    for (int i = 0; i < kPieces; i++) {
      const int src = i * (64 / kPieces) + lane / kPieces;
      char* b = (char*)__shfl((unsigned long long)mine, src);
      dst[i] = b ? b + 16 * (lane % kPieces) : nullptr;
      src_rounds[i] = __shfl(my_rounds, src);
    }
    uint32_t* row = rows + lane * RegStage<CW>::kRowWords;
    for (uint64_t rd = 0; rd < rounds; rd++) {
      if (rd < my_rounds) {
#pragma unroll
        for (int q = 0; q < kPieces; q++) {
          uint4 v;
          if (DT == PRAND_F64) {
            const double a = G::f64(G::next(r)), b = G::f64(G::next(r));
            const uint64_t ua = __double_as_longlong(a), ub = __double_as_longlong(b);
            v = make_uint4((uint32_t)ua, (uint32_t)(ua >> 32), (uint32_t)ub, (uint32_t)(ub >> 32));
          } else if (DT == PRAND_F32) {
            const uint32_t a = G::next(r), b = G::next(r), c = G::next(r), d = G::next(r);
            v = make_uint4(__float_as_uint((float)(a >> 8) * 0x1p-24f), __float_as_uint((float)(b >> 8) * 0x1p-24f),
                           __float_as_uint((float)(c >> 8) * 0x1p-24f), __float_as_uint((float)(d >> 8) * 0x1p-24f));
          } else {
            const uint32_t a = G::next(r), b = G::next(r), c = G::next(r), d = G::next(r);
            v = make_uint4(a, b, c, d);
          }
          *(uint4*)(row + 4 * q) = v;
        }
      }
      wave_lds_sync();
      const uint64_t adv = rd * per * es;
#pragma unroll
      for (int i = 0; i < kPieces; i++) {
        const int src = i * (64 / kPieces) + lane / kPieces;
        const uint4 v = *(const uint4*)(rows + src * RegStage<CW>::kRowWords + 4 * (lane % kPieces));
        if (dst[i] && rd < src_rounds[i]) store_out16<DT, (CW >= 32)>(dst[i] + adv, v);
      }
      wave_lds_sync();
    }
  }
  if (live) {
    for (uint64_t i = my_rounds * per; i < len; i++) {
      const uint32_t w = G::next(r);
      put_word<DT>(out, i, w, DT == PRAND_F64 ? G::f64(w) : 0.0);
    }
    if (sout) *sout = G::save(r);
  }
}

// Many streams: lane gid owns section gid & (nsec - 1) of stream
// gid >> nsec_log2; the sections of a stream cover
// [j * seclen, min((j + 1) * seclen, n)) and sit in one wavefront (nsec <= 64),
// so the state read of every section precedes the write-back of the last.
// With sectab (the section-start table of seclen), section j > 0 starts from
// row j - 1 of it, else from ladder jumps.
template <class G, int DT, int CW>
__global__ void __launch_bounds__(256) regstream_kernel(const typename G::State* sin, typename G::State* sout,
                                                        uint32_t count, uint64_t n, int nsec_log2, uint64_t seclen,
                                                        void* __restrict__ out, const uint32_t* __restrict__ ladder,
                                                        const uint32_t* __restrict__ sectab, int coalesce) {
  __shared__ __align__(16) uint32_t stage[4][RegStage<CW>::kWaveWords];
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t nsec = 1ull << nsec_log2;
  const uint64_t jlast = (n == 0) ? 0 : (n - 1) / seclen;
  const uint64_t s = gid >> nsec_log2, j = gid & (nsec - 1);
  const uint64_t start = j * seclen;
  const bool live = s < count && j <= jlast;
  const uint64_t len = live ? ((j == jlast) ? n - start : seclen) : 0;
  constexpr int es = (DT == PRAND_F64) ? 8 : 4;
  void* o = (char*)out + (s * n + start) * es;
  const uint32_t* sec_mat = (sectab && j) ? sectab + (j - 1) * G::kSectionWords : nullptr;
  regstream_wave<G, DT, CW>(stage[threadIdx.x >> 6], live, sin + (live ? s : 0), start, len, o,
                            (live && j == jlast) ? sout + s : nullptr, coalesce != 0, ladder, sec_mat);
}

// CW of the register-state kernels: 32 unless PRAND_REG_CHUNK_WORDS=16
inline int regstream_chunk_words() {
  static int cw = -1;
  if (cw < 0) {
    const char* e = getenv("PRAND_REG_CHUNK_WORDS");
    cw = (e && atoi(e) == 16) ? 16 : 32;
  }
  return cw;
}

template <class G, int CW>
hipError_t launch_regstream_cw(const typename G::State* sin, typename G::State* sout, uint32_t count, uint64_t n,
                               int nsec_log2, uint64_t seclen, int dtype, void* out, const uint32_t* ladder,
                               const uint32_t* sectab, hipStream_t st) {
  const uint64_t lanes = (uint64_t)count << nsec_log2;
  const uint32_t blocks = (uint32_t)((lanes + 255) / 256);
  // transposed 16-byte stores need every section start 16-byte aligned
  const uint64_t es = dtype == PRAND_F64 ? 8 : 4;
  const int coalesce = ((uintptr_t)out % 16 == 0) && ((n * es) % 16 == 0) && ((seclen * es) % 16 == 0);
  switch (dtype) {
    case PRAND_U32:
      hipLaunchKernelGGL((regstream_kernel<G, PRAND_U32, CW>), dim3(blocks), dim3(256), 0, st, sin, sout, count, n,
                         nsec_log2, seclen, out, ladder, sectab, coalesce);
      break;
    case PRAND_F32:
      hipLaunchKernelGGL((regstream_kernel<G, PRAND_F32, CW>), dim3(blocks), dim3(256), 0, st, sin, sout, count, n,
                         nsec_log2, seclen, out, ladder, sectab, coalesce);
      break;
    default:
      hipLaunchKernelGGL((regstream_kernel<G, PRAND_F64, CW>), dim3(blocks), dim3(256), 0, st, sin, sout, count, n,
                         nsec_log2, seclen, out, ladder, sectab, coalesce);
      break;
  }
  return hipGetLastError();
}

template <class G>
hipError_t launch_regstream(const typename G::State* sin, typename G::State* sout, uint32_t count, uint64_t n,
                            int nsec_log2, uint64_t seclen, int dtype, void* out, const uint32_t* ladder,
                            const uint32_t* sectab, hipStream_t st) {
  if (regstream_chunk_words() == 16)
    return launch_regstream_cw<G, 16>(sin, sout, count, n, nsec_log2, seclen, dtype, out, ladder, sectab, st);
  return launch_regstream_cw<G, 32>(sin, sout, count, n, nsec_log2, seclen, dtype, out, ladder, sectab, st);
}

}  // namespace prand
