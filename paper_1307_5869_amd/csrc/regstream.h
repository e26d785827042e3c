// Many-stream generation for generators whose whole state fits in a lane's
// registers (MRG32K3A, LFSR113).
//
// Lane gid owns section gid & (nsec - 1) of stream gid >> nsec_log2; the
// sections of a stream cover [j * seclen, min((j + 1) * seclen, n)) and start
// by jumping j * seclen ahead.  Each lane's outputs are contiguous in memory
// but 64 lanes write 64 different places, so a lane produces its outputs in
// chunks of CW words (CW = 32: 128 bytes, 32 u32/f32 or 16 f64 values), parks
// them in LDS, and the wavefront stores them transposed: in each store
// instruction the CW/4 consecutive lanes of a group write the 16-byte pieces
// of one chunk (CW = 32: eight whole 128-byte lines per instruction; CW = 16
// halves the LDS footprint and doubles occupancy with 64-byte segments).
// Rounds run while every live lane of the wavefront still has a full chunk
// to write; the rest of a section is stored lane by lane.  The lane whose
// section ends at n writes the advanced state to sout.
#pragma once

#include <cstdlib>

#include "prand_impl.h"

namespace prand {


// Order this wavefront's LDS writes before its later LDS reads (and reads
// before later writes).  The staging rows are private to the wavefront, so
// no workgroup barrier is needed -- and none may be used, since wavefronts of
// one workgroup can run different numbers of rounds.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int DT>
__device__ __forceinline__ void put_word(void* out, uint64_t i, uint32_t w, double f64v) {
  if (DT == PRAND_U32) ((uint32_t*)out)[i] = w;
  else if (DT == PRAND_F32) ((float*)out)[i] = (float)(w >> 8) * 0x1p-24f;
  else ((double*)out)[i] = f64v;
}

// G: State, Regs, static load(State) -> Regs, static save(Regs) -> State,
// static jump(State&, uint64_t distance, const uint32_t* ladder),
// static next(Regs&) -> uint32_t word, static f64(uint32_t) -> double.
template <class G, int DT, int CW>
__global__ void __launch_bounds__(256) regstream_kernel(const typename G::State* sin, typename G::State* sout,
                                                        uint32_t count, uint64_t n, int nsec_log2, uint64_t seclen,
                                                        void* __restrict__ out, const uint32_t* __restrict__ ladder,
                                                        int coalesce) {
  constexpr int kRowWords = CW + 4;   // padded LDS row, 16-byte aligned
  constexpr int kPieces = CW / 4;     // 16-byte pieces per chunk
  __shared__ __align__(16) uint32_t stage[256 / 64][64 * kRowWords];
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  uint32_t* rows = stage[threadIdx.x >> 6];
  const uint64_t nsec = 1ull << nsec_log2;
  const uint64_t jlast = (n == 0) ? 0 : (n - 1) / seclen;
  auto section = [&](uint64_t g, uint64_t& s, uint64_t& j, uint64_t& start, uint64_t& len) -> bool {
    s = g >> nsec_log2;
    j = g & (nsec - 1);
    start = j * seclen;
    len = (j == jlast) ? n - start : seclen;
    return s < count && j <= jlast;
  };
  uint64_t s, j, start, len;
  const bool live = section(gid, s, j, start, len);
  typename G::State st = {};
  if (live) {
    st = sin[s];
    if (start) G::jump(st, start, ladder);
  }
  typename G::Regs r = G::load(st);
  constexpr int per = (DT == PRAND_F64) ? CW / 2 : CW;   // values per chunk
  constexpr int es = (DT == PRAND_F64) ? 8 : 4;
  // full chunks every live lane of this wavefront can still write
  uint64_t my_rounds = live ? len / per : ~0ull;
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t other = __shfl_xor(my_rounds, o);
    my_rounds = other < my_rounds ? other : my_rounds;
  }
  const uint64_t rounds = (my_rounds == ~0ull || !coalesce) ? 0 : my_rounds;
  const uint64_t gid0 = gid - lane;
  char* const obytes = (char*)out;
  for (uint64_t rd = 0; rd < rounds; rd++) {
    uint32_t* row = rows + lane * kRowWords;
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
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < kPieces; i++) {
      const int src = i * (64 / kPieces) + lane / kPieces, piece = lane % kPieces;
      uint64_t ss, sj, sstart, slen;
      const bool slive = section(gid0 + src, ss, sj, sstart, slen);
      const uint4 v = *(const uint4*)(rows + src * kRowWords + 4 * piece);
      if (slive) {
        const uint64_t byte = (ss * n + sstart + rd * per) * es + 16 * piece;
        *(uint4*)(obytes + byte) = v;
      }
    }
    wave_lds_sync();
  }
  if (live) {
    for (uint64_t i = rounds * per; i < len; i++) {
      const uint32_t w = G::next(r);
      put_word<DT>(out, s * n + start + i, w, DT == PRAND_F64 ? G::f64(w) : 0.0);
    }
    if (j == jlast) sout[s] = G::save(r);
  }
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
                            hipStream_t st) {
  const uint64_t lanes = (uint64_t)count << nsec_log2;
  const uint32_t blocks = (uint32_t)((lanes + 255) / 256);
  // transposed 16-byte stores need every section start 16-byte aligned
  const uint64_t es = dtype == PRAND_F64 ? 8 : 4;
  const int coalesce = ((uintptr_t)out % 16 == 0) && ((n * es) % 16 == 0) && ((seclen * es) % 16 == 0);
  switch (dtype) {
    case PRAND_U32:
      hipLaunchKernelGGL((regstream_kernel<G, PRAND_U32, CW>), dim3(blocks), dim3(256), 0, st, sin, sout, count, n,
                         nsec_log2, seclen, out, ladder, coalesce);
      break;
    case PRAND_F32:
      hipLaunchKernelGGL((regstream_kernel<G, PRAND_F32, CW>), dim3(blocks), dim3(256), 0, st, sin, sout, count, n,
                         nsec_log2, seclen, out, ladder, coalesce);
      break;
    default:
      hipLaunchKernelGGL((regstream_kernel<G, PRAND_F64, CW>), dim3(blocks), dim3(256), 0, st, sin, sout, count, n,
                         nsec_log2, seclen, out, ladder, coalesce);
      break;
  }
  return hipGetLastError();
}

template <class G>
hipError_t launch_regstream(const typename G::State* sin, typename G::State* sout, uint32_t count, uint64_t n,
                            int nsec_log2, uint64_t seclen, int dtype, void* out, const uint32_t* ladder,
                            hipStream_t st) {
  if (regstream_chunk_words() == 16)
    return launch_regstream_cw<G, 16>(sin, sout, count, n, nsec_log2, seclen, dtype, out, ladder, st);
  return launch_regstream_cw<G, 32>(sin, sout, count, n, nsec_log2, seclen, dtype, out, ladder, st);
}

}  // namespace prand
