/*
 * prand_device.h -- header-only HIP device functions for drawing numbers
 * inside user kernels, one state per thread, with the eleven generators of
 * Barash & Shchur, "PRAND: GPU accelerated parallel random number generation
 * library", Comput. Phys. Commun. 185 (2014) 1343.
 *
 * This is the paper's single-threaded generation on the GPU (section
 * "Single-threaded generation", and the device functions rng_generate_ and
 * rng_generate_uniform_float_ of section "Header files"): a thread holds a
 * whole generator state and advances it one output at a time, so a kernel
 * uses the numbers where it draws them, with no array in HBM between the
 * generator and the consumer.  The states are the plain-old-data blobs of
 * prand.h (same layout, byte for byte), so a state initialised by the
 * library (prand_init_streams_dev, prand_seed_dev, prand_skipahead_dev) can
 * be handed to a user kernel, advanced there, and continued by the library's
 * bulk calls, and the other way round; the outputs are those of the bulk
 * calls.  Per output word:
 *   MT19937   the tempered word; every 624th call renews the 624-word block
 *             in place (the thread runs the whole twist)
 *   MRG32K3A  z = (x - y) mod m1 in [1, m1] (L'Ecuyer's combination)
 *   LFSR113   XOR of the four components' words (relations lfsrRel1 and
 *             lfsrOutput of the paper)
 *   GM/GQ     every element steps x^(n+1) = k x^(n) - q x^(n-1) mod g
 *             (recurrence rec1, Table 2); the digits floor(2^v x / g),
 *             element 0 first and most significant first, form the word.
 *             GQ58.3 yields 36 bits per step, 9 words per block of 8 steps:
 *             the state stays at the start of its block and `off` counts the
 *             block's words already used.
 * Conversions: float (w >> 8) * 2^-24, double w * 2^-32, MRG32K3A double
 * z * RN(1/(m1 + 1)) -- the values the bulk calls write.
 *
 * All arithmetic is exact integer arithmetic (64-bit, and a 128-bit product
 * for GM61); the functions favour plain code over speed (bulk generation is
 * the library's kernels' job).  They compile for the host as well.
 * State pointers may point to global memory, LDS or registers (a local
 * copy).  A state must not be advanced by two threads at once.
 */
#ifndef PRAND_DEVICE_H
#define PRAND_DEVICE_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "prand.h"

/* every function also compiles for the host (the same code then runs on the
   CPU, e.g. to continue a stream there) */
#define PRAND_FN __host__ __device__ inline

/* the state blobs of prand.h as C structs */
typedef struct {
  uint32_t mt[624];
  uint32_t idx;      /* next word of mt[] to temper; 624: the block is used up */
  uint32_t pad[3];
} prand_mt19937_state;
typedef struct {
  uint32_t x[3];     /* x_n, x_{n-1}, x_{n-2} mod m1 */
  uint32_t y[3];     /* y_n, y_{n-1}, y_{n-2} mod m2 */
} prand_mrg32k3a_state;
typedef struct {
  uint32_t z[4];
} prand_lfsr113_state;
typedef struct {
  uint64_t xp[32];   /* x^(n-1) of element i (i < s), exact residue mod g */
  uint64_t xc[32];   /* x^(n) */
  uint32_t off;      /* GQ58.3: words of the current 8-step block used, else 0 */
  uint32_t pad;
} prand_gm_state;

/* ---------------------------------------------------------------- MT19937 */
PRAND_FN uint32_t prand_mt19937_next(prand_mt19937_state* s) {
  if (s->idx >= 624u) {
    for (int j = 0; j < 624; j++) {
      const uint32_t y = (s->mt[j] & 0x80000000u) | (s->mt[j == 623 ? 0 : j + 1] & 0x7FFFFFFFu);
      const int m = j + 397 < 624 ? j + 397 : j + 397 - 624;
      s->mt[j] = s->mt[m] ^ (y >> 1) ^ ((y & 1u) ? 0x9908B0DFu : 0u);
    }
    s->idx = 0;
  }
  uint32_t y = s->mt[s->idx++];
  y ^= y >> 11;
  y ^= (y << 7) & 0x9D2C5680u;
  y ^= (y << 15) & 0xEFC60000u;
  return y ^ (y >> 18);
}

/* --------------------------------------------------------------- MRG32K3A */
PRAND_FN uint32_t prand_mrg32k3a_next(prand_mrg32k3a_state* s) {
  const uint64_t m1 = 4294967087ull, m2 = 4294944443ull;
  /* x_{n+1} = 1403580 x_{n-1} - 810728 x_{n-2} mod m1,
     y_{n+1} = 527612 y_n - 1370589 y_{n-2} mod m2 (sums below 2^54) */
  const uint64_t x = (1403580ull * s->x[1] + 810728ull * (m1 - s->x[2])) % m1;
  const uint64_t y = (527612ull * s->y[0] + 1370589ull * (m2 - s->y[2])) % m2;
  s->x[2] = s->x[1]; s->x[1] = s->x[0]; s->x[0] = (uint32_t)x;
  s->y[2] = s->y[1]; s->y[1] = s->y[0]; s->y[0] = (uint32_t)y;
  return (uint32_t)(x > y ? x - y : x + m1 - y);
}

/* ---------------------------------------------------------------- LFSR113 */
PRAND_FN uint32_t prand_lfsr113_comp(uint32_t z, uint32_t mask, int q, int k_s, int s) {
  return ((z & mask) << s) ^ (((z << q) ^ z) >> k_s);
}
PRAND_FN uint32_t prand_lfsr113_next(prand_lfsr113_state* s) {
  /* (k, q, s) = (31, 6, 18), (29, 2, 2), (28, 13, 7), (25, 3, 13) */
  s->z[0] = prand_lfsr113_comp(s->z[0], 0xFFFFFFFEu, 6, 13, 18);
  s->z[1] = prand_lfsr113_comp(s->z[1], 0xFFFFFFF8u, 2, 27, 2);
  s->z[2] = prand_lfsr113_comp(s->z[2], 0xFFFFFFF0u, 13, 21, 7);
  s->z[3] = prand_lfsr113_comp(s->z[3], 0xFFFFFF80u, 3, 12, 13);
  return s->z[0] ^ s->z[1] ^ s->z[2] ^ s->z[3];
}

/* ------------------------------------------------------------------ GM/GQ */
typedef struct {
  uint64_t k, q, g;  /* g = p 2^t */
  int v, s;          /* digit bits, ensemble size */
} prand_gm_params;

/* Table 2 parameters with the ensemble sizes of Table 5, gen = PRAND_GM19..PRAND_GQ58X4 */
PRAND_FN prand_gm_params prand_gm_params_of(int gen) {
  switch (gen) {
    case PRAND_GM19: return prand_gm_params{15, 28, 524287ull, 1, 32};
    case PRAND_GM29: return prand_gm_params{4, 2, 536870909ull, 1, 32};
    case PRAND_GM31: return prand_gm_params{11, 14, 2147483647ull, 1, 32};
    case PRAND_GM55: return prand_gm_params{256, 176, 16ull * 2251799813685119ull, 4, 8};
    case PRAND_GM61: return prand_gm_params{24, 74, 2305843009213693951ull, 1, 32};
    case PRAND_GQ58X1: return prand_gm_params{8, 48, 536870912ull * 536870909ull, 1, 32};
    case PRAND_GQ58X3: return prand_gm_params{8, 48, 536870912ull * 536870909ull, 3, 12};
    default: return prand_gm_params{8, 48, 536870912ull * 536870909ull, 4, 8};
  }
}

/* k xc - q xp mod g for residues xc, xp < g */
PRAND_FN uint64_t prand_gm_step_elem(const prand_gm_params& P, uint64_t xc, uint64_t xp) {
  if (P.g == 2305843009213693951ull) {
    /* GM61: the sum reaches 2^68; fold with 2^61 = 1 (mod 2^61 - 1) */
    const unsigned __int128 t = (unsigned __int128)P.k * xc + (unsigned __int128)P.q * (P.g - xp);
    const uint64_t lo = (uint64_t)t, hi = (uint64_t)(t >> 64);
    uint64_t r = (lo & P.g) + ((lo >> 61) | (hi << 3));
    r = (r & P.g) + (r >> 61);
    return r >= P.g ? r - P.g : r;
  }
  /* every other modulus: (k + q) g <= 432 g < 2^64, so the sum fits 64 bits */
  return (P.k * xc + P.q * (P.g - xp)) % P.g;
}

/* one ensemble step: advances every element, returns the s v digit bits
   (element 0 most significant) */
PRAND_FN uint64_t prand_gm_ensemble_step(const prand_gm_params& P, prand_gm_state* st) {
  uint64_t bits = 0;
  for (int i = 0; i < P.s; i++) {
    const uint64_t nx = prand_gm_step_elem(P, st->xc[i], st->xp[i]);
    st->xp[i] = st->xc[i];
    st->xc[i] = nx;
    bits = (bits << P.v) | ((nx << P.v) / P.g);   /* floor(2^v x / g); 2^v x < 2^63 */
  }
  return bits;
}

PRAND_FN uint32_t prand_gm_next(int gen, prand_gm_state* st) {
  const prand_gm_params P = prand_gm_params_of(gen);
  if (gen != PRAND_GQ58X3) return (uint32_t)prand_gm_ensemble_step(P, st);
  /* GQ58.3: word w of a block covers bits [32 w, 32 w + 32) of the block's
     288 bits (steps of 36 bits each); step a copy from the block start as
     far as that word needs */
  const uint32_t w = st->off;
  prand_gm_state tmp;
  for (int i = 0; i < 12; i++) { tmp.xp[i] = st->xp[i]; tmp.xc[i] = st->xc[i]; }
  const int first = (int)(32 * w) / 36, last = (int)(32 * w + 31) / 36;
  uint64_t acc = 0;   /* bits of steps first..last, at most 72 needed: two halves */
  uint64_t hi_bits = 0;
  for (int stp = 0; stp <= last; stp++) {
    const uint64_t b = prand_gm_ensemble_step(P, &tmp);
    if (stp == first) hi_bits = b;
    if (stp == last) acc = b;
  }
  uint32_t word;
  const int shift = (int)(32 * w) - 36 * first;   /* bit position of the word inside step `first` */
  if (first == last) {
    word = (uint32_t)(hi_bits >> (36 - shift - 32));
  } else {
    const int from_first = 36 - shift;             /* bits taken from step `first` */
    word = (uint32_t)(((hi_bits & ((1ull << from_first) - 1)) << (32 - from_first)) |
                      (acc >> (36 - (32 - from_first))));
  }
  if (w == 8) {   /* block used up: the state moves to the next block */
    for (int i = 0; i < 12; i++) { st->xp[i] = tmp.xp[i]; st->xc[i] = tmp.xc[i]; }
    st->off = 0;
  } else {
    st->off = w + 1;
  }
  return word;
}

/* ---------------------------------------------------------------- generic */
/* Next 32-bit output of generator `gen` from its state blob. */
PRAND_FN uint32_t prand_next(int gen, void* state) {
  switch (gen) {
    case PRAND_MT19937: return prand_mt19937_next((prand_mt19937_state*)state);
    case PRAND_MRG32K3A: return prand_mrg32k3a_next((prand_mrg32k3a_state*)state);
    case PRAND_LFSR113: return prand_lfsr113_next((prand_lfsr113_state*)state);
    default: return prand_gm_next(gen, (prand_gm_state*)state);
  }
}

/* the library's integer-to-float maps of a word of generator `gen` */
PRAND_FN float prand_word_to_float(uint32_t w) { return (float)(w >> 8) * 0x1p-24f; }
PRAND_FN double prand_word_to_double(int gen, uint32_t w) {
  return gen == PRAND_MRG32K3A ? (double)w * (1.0 / 4294967088.0) : (double)w * 0x1p-32;
}

/* rng_generate_uniform_float_ / _double_ of the paper: a number in [0, 1)
   ((0, 1) for MRG32K3A doubles) from the next word */
PRAND_FN float prand_uniform_float(int gen, void* state) {
  return prand_word_to_float(prand_next(gen, state));
}
PRAND_FN double prand_uniform_double(int gen, void* state) {
  return prand_word_to_double(gen, prand_next(gen, state));
}

#endif /* PRAND_DEVICE_H */
