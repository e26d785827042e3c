// Seeding (the paper's rng_init_ and its seeded form), one lane per state.
//   MT19937: init_genrand(seed) for seed < 2^32, else init_by_array over the
//            two 32-bit halves (Matsumoto-Nishimura reference seeding).
//   MRG32K3A: all six words = seed when 1 <= seed < m2; LFSR113: all four
//            words = seed when 128 <= seed < 2^32.
//   Otherwise, and for every GM/GQ element, SplitMix64 draws from a start
//   state that is the first SplitMix64 output from
//   seed ^ (0x9E3779B97F4A7C15 * (gen + 1)) (the tags are multiples of the
//   Weyl increment, so starting at seed ^ tag itself would make the draws of
//   one generator those of another shifted by a few): the top bits of a draw, rejected
//   until below the bound; an MRG triple or a GM element pair that is zero
//   (mod p) is drawn again; an LFSR word is redrawn until its top p bits are
//   not all zero.
// The same functions serve the device kernel and the host-only entry points.
#include "prand_impl.h"

namespace prand {
namespace {

__host__ __device__ inline uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t seed_start(uint64_t seed, int gen) {
  uint64_t t = seed ^ (0x9E3779B97F4A7C15ull * (uint64_t)(gen + 1));
  return splitmix64(t);
}
__host__ __device__ inline uint64_t draw_below(uint64_t& s, uint64_t bound) {
  const int nb = 64 - __builtin_clzll(bound - 1);   // bound >= 2
  for (;;) {
    const uint64_t r = splitmix64(s) >> (64 - nb);
    if (r < bound) return r;
  }
}

__host__ __device__ void seed_mt(MtState* st, uint64_t seed) {
  uint32_t* mt = st->mt;
  auto genrand = [&](uint32_t s) {
    mt[0] = s;
    for (uint32_t i = 1; i < 624; i++) mt[i] = 1812433253u * (mt[i - 1] ^ (mt[i - 1] >> 30)) + i;
  };
  if (seed <= 0xFFFFFFFFull) {
    genrand((uint32_t)seed);
  } else {
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    genrand(19650218u);
    int i = 1, j = 0;
    for (int k = 624; k > 0; k--) {
      mt[i] = (mt[i] ^ ((mt[i - 1] ^ (mt[i - 1] >> 30)) * 1664525u)) + key[j] + (uint32_t)j;
      i++; j++;
      if (i >= 624) { mt[0] = mt[623]; i = 1; }
      if (j >= 2) j = 0;
    }
    for (int k = 623; k > 0; k--) {
      mt[i] = (mt[i] ^ ((mt[i - 1] ^ (mt[i - 1] >> 30)) * 1566083941u)) - (uint32_t)i;
      i++;
      if (i >= 624) { mt[0] = mt[623]; i = 1; }
    }
    mt[0] = 0x80000000u;
  }
  st->idx = 624;
  st->pad[0] = st->pad[1] = st->pad[2] = 0;
}

__host__ __device__ void seed_mrg(MrgState* st, uint64_t seed) {
  if (seed >= 1 && seed < kMrgM2) {
    for (int i = 0; i < 3; i++) { st->x[i] = (uint32_t)seed; st->y[i] = (uint32_t)seed; }
    return;
  }
  uint64_t sm = seed_start(seed, PRAND_MRG32K3A);
  uint32_t x[3], y[3];
  do { for (int i = 0; i < 3; i++) x[i] = (uint32_t)draw_below(sm, kMrgM1); } while (!(x[0] | x[1] | x[2]));
  do { for (int i = 0; i < 3; i++) y[i] = (uint32_t)draw_below(sm, kMrgM2); } while (!(y[0] | y[1] | y[2]));
  for (int i = 0; i < 3; i++) { st->x[i] = x[i]; st->y[i] = y[i]; }
}

__host__ __device__ void seed_lfsr(LfsrState* st, uint64_t seed) {
  if (seed >= 128 && seed <= 0xFFFFFFFFull) {
    for (int c = 0; c < 4; c++) st->z[c] = (uint32_t)seed;
    return;
  }
  const int p[4] = {31, 29, 28, 25};
  uint64_t sm = seed_start(seed, PRAND_LFSR113);
  for (int c = 0; c < 4; c++) {
    const uint32_t top = 0xFFFFFFFFu << (32 - p[c]);
    uint32_t z;
    do z = (uint32_t)(splitmix64(sm) >> 32); while (!(z & top));
    st->z[c] = z;
  }
}

__host__ __device__ void seed_gm(int gen, GmState* st, uint64_t seed) {
  const GmParams& P = kGmParams[gen - PRAND_GM19];
  const uint64_t g = P.p << P.t;
  uint64_t sm = seed_start(seed, gen);
  for (int i = 0; i < 32; i++) {
    uint64_t a = 0, b = 0;
    if (i < P.s) {
      do {
        a = draw_below(sm, g);
        b = draw_below(sm, g);
      } while (a % P.p == 0 && b % P.p == 0);
    }
    st->xp[i] = a;
    st->xc[i] = b;
  }
  st->off = 0;
  st->pad = 0;
}

__host__ __device__ void seed_one(int gen, uint64_t seed, void* state) {
  switch (gen) {
    case PRAND_MT19937: seed_mt((MtState*)state, seed); break;
    case PRAND_MRG32K3A: seed_mrg((MrgState*)state, seed); break;
    case PRAND_LFSR113: seed_lfsr((LfsrState*)state, seed); break;
    default: seed_gm(gen, (GmState*)state, seed); break;
  }
}

__host__ __device__ inline size_t state_size(int gen) {
  return gen == PRAND_MT19937 ? sizeof(MtState)
         : gen == PRAND_MRG32K3A ? sizeof(MrgState)
         : gen == PRAND_LFSR113 ? sizeof(LfsrState)
                                : sizeof(GmState);
}

__global__ void __launch_bounds__(256) seed_kernel(int gen, const uint64_t* __restrict__ seeds, uint32_t count,
                                                   void* __restrict__ states) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  seed_one(gen, seeds[i], (char*)states + (size_t)i * state_size(gen));
}

}  // namespace

void seed_host(int gen, uint64_t seed, void* h_state) { seed_one(gen, seed, h_state); }

hipError_t launch_seed(int gen, const uint64_t* seeds, uint32_t count, void* states, hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(seed_kernel, dim3((count + 255) / 256), dim3(256), 0, st, gen, seeds, count, states);
  return hipGetLastError();
}

}  // namespace prand
