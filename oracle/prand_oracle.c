/*
 * prand_oracle.c -- plain, slow, obviously correct CPU reference ("the
 * oracle") for the eleven generators of Barash & Shchur, "PRAND: GPU
 * accelerated parallel random number generation library", Comput. Phys.
 * Commun. 185 (2014) 1343.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library; the product path never
 * does.  It shares no code, header, table or constant generator with the GPU
 * library: every constant below is restated from the paper (or, where the
 * paper defers to the cited definition of a generator, from that published
 * definition) and every derived object (the MT19937 characteristic
 * polynomial, matrix powers) is computed here by its own routines.
 *
 * Arithmetic is exact integer arithmetic (mod m, or over F2) with 128-bit
 * intermediates; the only floating-point steps are the fixed integer-to-float
 * maps, each a single IEEE operation on an exactly representable value.
 *
 * Readings taken where the paper is silent or garbled:
 *  - every generator steps first and then outputs;
 *  - MRG32K3A output word z = (x - y) mod m1 taken in [1, m1] (the paper's
 *    "(x_n + y_n) mod g" names no g; the cited definition uses the
 *    difference modulo m1);
 *  - LFSR113 output word = XOR of its four component words;
 *  - MT19937 is the standard 32-bit Mersenne twister with default seed 5489;
 *  - GM/GQ ensembles: s = threads per array section of the paper's table of
 *    launch shapes (32, 8 or 12 elements), digit = floor(2^v x / g), digits
 *    packed element 0 first, most significant bit first, into consecutive
 *    32-bit words (GQ58.3: 36 bits per step, 9 words per 8 steps);
 *  - seeds: SplitMix64 expansion where a seed is not used verbatim (below);
 *  - block-splitting block lengths L are powers of two no smaller than the
 *    sequence lengths of the paper's stream table.
 *  - seed expansion: SplitMix64 draws from a start state that is the first
 *    SplitMix64 output of seed ^ (increment * (generator + 1)); pinned by its
 *    tests against an independent implementation of the SplitMix64 output
 *    function and the closed form of its increment.
 * Parity unpinned: the GM/GQ digit packing (the paper does not give it; only
 * internal consistency can be checked).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* generator, dtype and variant numbering (a fixed interface) */
enum {
  OR_MT19937 = 0, OR_MRG32K3A = 1, OR_LFSR113 = 2,
  OR_GM19 = 3, OR_GM29 = 4, OR_GM31 = 5, OR_GM55 = 6, OR_GM61 = 7,
  OR_GQ58X1 = 8, OR_GQ58X3 = 9, OR_GQ58X4 = 10, OR_NGEN = 11
};
enum { OR_U32 = 0, OR_F32 = 1, OR_F64 = 2 };
enum { OR_VAR_DEFAULT = 0, OR_VAR_SEQ = 1, OR_VAR_SHORT = 2, OR_VAR_MEDIUM = 3, OR_VAR_LONG = 4 };
#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_EUNSUPPORTED (-2)
#define OR_ERANGE (-3)
#define OR_ENOMEM (-5)

/* ------------------------------------------------------------------------ */
/* 512-bit unsigned distances, little-endian 64-bit limbs                   */
/* ------------------------------------------------------------------------ */
#define NLIMB 8
typedef struct { uint64_t w[NLIMB]; } big;

static int big_load(big* b, const uint64_t* limbs, int n) {
  if (n < 0 || n > NLIMB || (n > 0 && !limbs)) return OR_EINVAL;
  memset(b, 0, sizeof *b);
  for (int i = 0; i < n; i++) b->w[i] = limbs[i];
  return OR_OK;
}
static int big_bit(const big* b, int i) { return (int)((b->w[i >> 6] >> (i & 63)) & 1u); }
static int big_nbits(const big* b) {
  for (int i = NLIMB * 64 - 1; i >= 0; i--) if (big_bit(b, i)) return i + 1;
  return 0;
}
static int big_is_zero(const big* b) { return big_nbits(b) == 0; }
/* b += a; returns carry out */
static int big_add_small(big* b, uint64_t a) {
  for (int i = 0; i < NLIMB && a; i++) {
    uint64_t s = b->w[i] + a;
    a = (s < b->w[i]) ? 1 : 0;
    b->w[i] = s;
  }
  return a != 0;
}
/* b -= a, requires b >= a */
static void big_sub_small(big* b, uint64_t a) {
  for (int i = 0; i < NLIMB && a; i++) {
    uint64_t old = b->w[i];
    b->w[i] = old - a;
    a = (old < a) ? 1 : 0;
  }
}
/* b *= m; returns nonzero on overflow */
static int big_mul_small(big* b, uint64_t m) {
  uint64_t carry = 0;
  for (int i = 0; i < NLIMB; i++) {
    u128 t = (u128)b->w[i] * m + carry;
    b->w[i] = (uint64_t)t;
    carry = (uint64_t)(t >> 64);
  }
  return carry != 0;
}
/* b = b / d, returns b mod d */
static uint64_t big_divmod_small(big* b, uint64_t d) {
  u128 r = 0;
  for (int i = NLIMB - 1; i >= 0; i--) {
    u128 cur = (r << 64) | b->w[i];
    b->w[i] = (uint64_t)(cur / d);
    r = cur % d;
  }
  return (uint64_t)r;
}
static int big_le_small(const big* b, uint64_t a) {
  for (int i = 1; i < NLIMB; i++) if (b->w[i]) return 0;
  return b->w[0] <= a;
}

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea & Flood 2014; Vigna's published constants):      */
/* the seed expander used wherever a seed is not taken verbatim.            */
/* ------------------------------------------------------------------------ */
static uint64_t splitmix64(uint64_t* s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static uint64_t seed_tag(int gen) { return 0x9E3779B97F4A7C15ULL * (uint64_t)(gen + 1); }
/* start state of a seed's expansion: the first SplitMix64 output from
   seed ^ tag(gen).  (Starting at seed ^ tag(gen) itself would put the start
   states of different generators on the Weyl sequence the draws walk along,
   since the tags are multiples of its increment: for most seeds the draws of
   one generator would be those of another shifted by a few places.) */
static uint64_t seed_start(uint64_t seed, int gen) {
  uint64_t t = seed ^ seed_tag(gen);
  return splitmix64(&t);
}
/* uniform in [0, bound), bound >= 2: top bits of a draw, rejected when >= bound */
static uint64_t draw_below(uint64_t* s, uint64_t bound) {
  int nb = 64 - __builtin_clzll(bound - 1);
  for (;;) {
    uint64_t r = splitmix64(s) >> (64 - nb);
    if (r < bound) return r;
  }
}

/* ------------------------------------------------------------------------ */
/* fixed integer -> float maps                                              */
/* ------------------------------------------------------------------------ */
static float word_to_f32(uint32_t w) { return (float)(w >> 8) * 0x1p-24f; }
static double word_to_f64(uint32_t w) { return (double)w * 0x1p-32; }

/* ======================================================================== */
/* MRG32K3A: X_{n+1} = A X_n mod m1, Y_{n+1} = B Y_n mod m2 with            */
/* X_n = (x_n, x_{n-1}, x_{n-2}), A = ((0 a b)(1 0 0)(0 1 0)),               */
/* B = ((c 0 d)(1 0 0)(0 1 0)) -- paper, section on jumping ahead for       */
/* MRG32K3A.  State words: x_n, x_{n-1}, x_{n-2}, y_n, y_{n-1}, y_{n-2}.    */
/* ======================================================================== */
static const uint64_t MRG_M1 = 4294967087ULL;   /* 2^32 - 209   */
static const uint64_t MRG_M2 = 4294944443ULL;   /* 2^32 - 22853 */
static const int64_t MRG_A = 1403580, MRG_B = -810728, MRG_C = 527612, MRG_D = -1370589;

typedef struct { uint32_t x[3]; uint32_t y[3]; } or_mrg;

static uint64_t mod_i64(int64_t v, uint64_t m) {
  int64_t r = v % (int64_t)m;
  return (uint64_t)(r < 0 ? r + (int64_t)m : r);
}

static uint32_t mrg_next(or_mrg* s) {
  uint64_t xn = mod_i64(MRG_A * (int64_t)s->x[1] + MRG_B * (int64_t)s->x[2], MRG_M1);
  uint64_t yn = mod_i64(MRG_C * (int64_t)s->y[0] + MRG_D * (int64_t)s->y[2], MRG_M2);
  s->x[2] = s->x[1]; s->x[1] = s->x[0]; s->x[0] = (uint32_t)xn;
  s->y[2] = s->y[1]; s->y[1] = s->y[0]; s->y[0] = (uint32_t)yn;
  uint64_t z = (xn + MRG_M1 - yn) % MRG_M1;   /* yn < m2 < m1 */
  return (uint32_t)(z == 0 ? MRG_M1 : z);
}
static double mrg_to_f64(uint32_t z) { return (double)z * (1.0 / 4294967088.0); }

typedef struct { uint64_t a[3][3]; } m3;
static m3 m3_mul(const m3* P, const m3* Q, uint64_t m) {
  m3 R;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      u128 acc = 0;
      for (int k = 0; k < 3; k++) acc += (u128)P->a[i][k] * Q->a[k][j];
      R.a[i][j] = (uint64_t)(acc % m);
    }
  return R;
}
static m3 m3_pow(const m3* M, const big* N, uint64_t m) {
  m3 R; memset(&R, 0, sizeof R);
  for (int i = 0; i < 3; i++) R.a[i][i] = 1 % m;
  m3 P = *M;
  int nb = big_nbits(N);
  for (int i = 0; i < nb; i++) {
    if (big_bit(N, i)) R = m3_mul(&R, &P, m);
    P = m3_mul(&P, &P, m);
  }
  return R;
}
static void m3_apply(const m3* M, uint32_t v[3], uint64_t m) {
  uint64_t r[3];
  for (int i = 0; i < 3; i++) {
    u128 acc = 0;
    for (int k = 0; k < 3; k++) acc += (u128)M->a[i][k] * v[k];
    r[i] = (uint64_t)(acc % m);
  }
  for (int i = 0; i < 3; i++) v[i] = (uint32_t)r[i];
}
static m3 mrg_matrix_A(void) {
  m3 A; memset(&A, 0, sizeof A);
  A.a[0][1] = mod_i64(MRG_A, MRG_M1); A.a[0][2] = mod_i64(MRG_B, MRG_M1);
  A.a[1][0] = 1; A.a[2][1] = 1;
  return A;
}
static m3 mrg_matrix_B(void) {
  m3 B; memset(&B, 0, sizeof B);
  B.a[0][0] = mod_i64(MRG_C, MRG_M2); B.a[0][2] = mod_i64(MRG_D, MRG_M2);
  B.a[1][0] = 1; B.a[2][1] = 1;
  return B;
}
static void mrg_skip(or_mrg* s, const big* N) {
  m3 A = mrg_matrix_A(), B = mrg_matrix_B();
  m3 An = m3_pow(&A, N, MRG_M1), Bn = m3_pow(&B, N, MRG_M2);
  m3_apply(&An, s->x, MRG_M1);
  m3_apply(&Bn, s->y, MRG_M2);
}
static void mrg_seed(or_mrg* s, uint64_t seed) {
  if (seed >= 1 && seed < MRG_M2) {
    for (int i = 0; i < 3; i++) { s->x[i] = (uint32_t)seed; s->y[i] = (uint32_t)seed; }
    return;
  }
  uint64_t sm = seed_start(seed, OR_MRG32K3A);
  do { for (int i = 0; i < 3; i++) s->x[i] = (uint32_t)draw_below(&sm, MRG_M1); }
  while (!s->x[0] && !s->x[1] && !s->x[2]);
  do { for (int i = 0; i < 3; i++) s->y[i] = (uint32_t)draw_below(&sm, MRG_M2); }
  while (!s->y[0] && !s->y[1] && !s->y[2]);
}

/* ======================================================================== */
/* LFSR113: four shift-register sequences x_n = x_{n-p} + x_{n-p+q} mod 2    */
/* with output word u_n = sum_{i=1..32} x_{ns+i-1} 2^{-i}; (p,q,s) =          */
/* (31,6,18), (29,2,2), (28,13,7), (25,3,13) -- paper, section on jumping   */
/* ahead for LFSR113, relations lfsrRel1 and lfsrOutput.  One step of a     */
/* component maps the 32-bit window (x_{ns}..x_{ns+31}) to the next one:   */
/* the top p-s bits are the old window shifted by s, the rest follow from   */
/* the recurrence applied to the old window (valid since p >= s+q).         */
/* ======================================================================== */
static const int LF_P[4] = {31, 29, 28, 25};
static const int LF_Q[4] = {6, 2, 13, 3};
static const int LF_S[4] = {18, 2, 7, 13};

typedef struct { uint32_t z[4]; } or_lfsr;

static uint32_t lfsr_comp_step(uint32_t z, int p, int q, int s) {
  uint32_t topmask = 0xFFFFFFFFu << (32 - p);       /* the p bits x_{ns}..x_{ns+p-1} */
  uint32_t fresh = ((z << q) ^ z) >> (p - s);        /* x_{ns+i} + x_{ns+i+q} = x_{ns+i+p} */
  return ((z & topmask) << s) ^ fresh;
}
static uint32_t lfsr_next(or_lfsr* st) {
  uint32_t w = 0;
  for (int c = 0; c < 4; c++) {
    st->z[c] = lfsr_comp_step(st->z[c], LF_P[c], LF_Q[c], LF_S[c]);
    w ^= st->z[c];
  }
  return w;
}
/* a 32x32 matrix over F2 stored by columns: col[j] = image of bit j */
typedef struct { uint32_t col[32]; } f2m;
static uint32_t f2m_apply(const f2m* M, uint32_t v) {
  uint32_t r = 0;
  for (int j = 0; j < 32; j++) if ((v >> j) & 1u) r ^= M->col[j];
  return r;
}
static f2m f2m_mul(const f2m* P, const f2m* Q) {  /* P after Q */
  f2m R;
  for (int j = 0; j < 32; j++) R.col[j] = f2m_apply(P, Q->col[j]);
  return R;
}
static uint32_t lfsr_comp_jump(uint32_t z, int p, int q, int s, const big* N) {
  f2m T;
  for (int j = 0; j < 32; j++) T.col[j] = lfsr_comp_step(1u << j, p, q, s);
  f2m R;
  for (int j = 0; j < 32; j++) R.col[j] = 1u << j;
  int nb = big_nbits(N);
  for (int i = 0; i < nb; i++) {
    if (big_bit(N, i)) R = f2m_mul(&T, &R);
    T = f2m_mul(&T, &T);
  }
  return f2m_apply(&R, z);
}
static void lfsr_skip(or_lfsr* st, const big* N) {
  for (int c = 0; c < 4; c++) st->z[c] = lfsr_comp_jump(st->z[c], LF_P[c], LF_Q[c], LF_S[c], N);
}
static void lfsr_seed(or_lfsr* st, uint64_t seed) {
  if (seed >= 128 && seed <= 0xFFFFFFFFULL) {
    for (int c = 0; c < 4; c++) st->z[c] = (uint32_t)seed;
    return;
  }
  uint64_t sm = seed_start(seed, OR_LFSR113);
  for (int c = 0; c < 4; c++) {
    uint32_t topmask = 0xFFFFFFFFu << (32 - LF_P[c]);
    do st->z[c] = (uint32_t)(splitmix64(&sm) >> 32); while (!(st->z[c] & topmask));
  }
}

/* ======================================================================== */
/* MT19937 (Matsumoto & Nishimura): w=32, n=624, m=397, r=31,                */
/* a=0x9908B0DF, tempering (11, 7/0x9D2C5680, 15/0xEFC60000, 18).  Its       */
/* linear transition Y_{n+1} = A Y_n over F2 and the jump                    */
/* A^v Y = g_v(A) Y with g_v(x) = x^v mod phi(x) follow the paper's section  */
/* on jumping ahead for MT19937 (equation g_v).                              */
/* ======================================================================== */
#define MT_N 624
#define MT_M 397
#define MT_DEG 19937
#define PW 312                       /* 64-bit words holding 19968 >= 19937 bits */

typedef struct { uint32_t mt[MT_N]; uint32_t mti; uint32_t pad[3]; } or_mt;

static void mt_init_genrand(or_mt* st, uint32_t s) {
  memset(st, 0, sizeof *st);
  st->mt[0] = s;
  for (uint32_t i = 1; i < MT_N; i++)
    st->mt[i] = 1812433253u * (st->mt[i - 1] ^ (st->mt[i - 1] >> 30)) + i;
  st->mti = MT_N;
}
static void mt_init_by_array(or_mt* st, const uint32_t* key, int len) {
  mt_init_genrand(st, 19650218u);
  uint32_t* mt = st->mt;
  int i = 1, j = 0;
  for (int k = (MT_N > len ? MT_N : len); k > 0; k--) {
    mt[i] = (mt[i] ^ ((mt[i - 1] ^ (mt[i - 1] >> 30)) * 1664525u)) + key[j] + (uint32_t)j;
    i++; j++;
    if (i >= MT_N) { mt[0] = mt[MT_N - 1]; i = 1; }
    if (j >= len) j = 0;
  }
  for (int k = MT_N - 1; k > 0; k--) {
    mt[i] = (mt[i] ^ ((mt[i - 1] ^ (mt[i - 1] >> 30)) * 1566083941u)) - (uint32_t)i;
    i++;
    if (i >= MT_N) { mt[0] = mt[MT_N - 1]; i = 1; }
  }
  mt[0] = 0x80000000u;
  st->mti = MT_N;
}
/* x_{j+n} = x_{j+m} ^ ((upper(x_j) | lower(x_{j+1})) A): one raw word */
static uint32_t mt_recur(uint32_t xj, uint32_t xj1, uint32_t xjm) {
  uint32_t y = (xj & 0x80000000u) | (xj1 & 0x7FFFFFFFu);
  return xjm ^ (y >> 1) ^ ((y & 1u) ? 0x9908B0DFu : 0u);
}
static void mt_twist(or_mt* st) {
  /* in place: indices that wrap refer to words already renewed, which are the
     newer sequence words the recurrence asks for */
  for (int j = 0; j < MT_N; j++)
    st->mt[j] = mt_recur(st->mt[j], st->mt[(j + 1) % MT_N], st->mt[(j + MT_M) % MT_N]);
  st->mti = 0;
}
static uint32_t mt_temper(uint32_t y) {
  y ^= y >> 11;
  y ^= (y << 7) & 0x9D2C5680u;
  y ^= (y << 15) & 0xEFC60000u;
  y ^= y >> 18;
  return y;
}
static uint32_t mt_next(or_mt* st) {
  if (st->mti >= MT_N) mt_twist(st);
  return mt_temper(st->mt[st->mti++]);
}
static void mt_seed(or_mt* st, uint64_t seed) {
  if (seed <= 0xFFFFFFFFULL) { mt_init_genrand(st, (uint32_t)seed); return; }
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  mt_init_by_array(st, key, 2);
}

/* --- polynomials over F2: bit i of a word array = coefficient of x^i --- */
static int pbit(const uint64_t* a, int i) { return (int)((a[i >> 6] >> (i & 63)) & 1u); }
static void pflip(uint64_t* a, int i) { a[i >> 6] ^= 1ULL << (i & 63); }

static uint64_t g_phi[PW];   /* phi(x) minus its leading term x^19937 */
static int g_phi_ready = 0;

/* Berlekamp-Massey on 2*19937 output bits (bit 0 of successive outputs from
   the default state).  The minimal polynomial of that sequence is the
   characteristic polynomial of A because the latter is irreducible. */
static int mt_compute_phi(void) {
  const int n = 2 * MT_DEG;
  const int nw = n / 64 + 2;
  uint64_t* s = (uint64_t*)calloc(nw, 8);
  uint64_t* C = (uint64_t*)calloc(nw, 8);
  uint64_t* B = (uint64_t*)calloc(nw, 8);
  uint64_t* T = (uint64_t*)calloc(nw, 8);
  if (!s || !C || !B || !T) { free(s); free(C); free(B); free(T); return OR_ENOMEM; }
  or_mt st;
  mt_init_genrand(&st, 5489u);
  for (int i = 0; i < n; i++) if (mt_next(&st) & 1u) pflip(s, i);
  C[0] = 1; B[0] = 1;
  int L = 0, m = 1, degB = 0;
  for (int i = 0; i < n; i++) {
    int d = pbit(s, i);
    for (int j = 1; j <= L; j++) d ^= pbit(C, j) & pbit(s, i - j);
    if (!d) { m++; continue; }
    memcpy(T, C, (size_t)nw * 8);
    for (int j = 0; j <= degB; j++) if (pbit(B, j)) pflip(C, j + m);   /* C += x^m B */
    if (2 * L <= i) {
      int oldL = L;
      L = i + 1 - L;
      memcpy(B, T, (size_t)nw * 8);
      degB = oldL;
      m = 1;
    } else {
      m++;
    }
  }
  int ok = (L == MT_DEG);
  if (ok) {
    /* phi(x) = x^L C(1/x): coefficient of x^i is c_{L-i} */
    memset(g_phi, 0, sizeof g_phi);
    for (int i = 0; i < MT_DEG; i++) if (pbit(C, MT_DEG - i)) pflip(g_phi, i);
    g_phi_ready = 1;
  }
  free(s); free(C); free(B); free(T);
  return ok ? OR_OK : OR_ERANGE;
}
static int mt_need_phi(void) { return g_phi_ready ? OR_OK : mt_compute_phi(); }

/* reduce a polynomial of degree < 2*19937 held in 2*PW+1 words modulo phi,
   top term first; phi = x^19937 + g_phi */
static void poly_reduce(uint64_t* a) {
  for (int d = 2 * MT_DEG - 2; d >= MT_DEG; d--) {
    if (!pbit(a, d)) continue;
    pflip(a, d);
    int sh = d - MT_DEG;
    for (int i = 0; i < MT_DEG; i++) if (pbit(g_phi, i)) pflip(a, i + sh);
  }
}
/* the bit-level reduction above is the obviously-correct version; the
   word-level one below does the same XOR of (g_phi << sh), 64 bits at a time */
static void poly_reduce_fast(uint64_t* a) {
  for (int d = 2 * MT_DEG - 2; d >= MT_DEG; d--) {
    if (!pbit(a, d)) continue;
    pflip(a, d);
    int sh = d - MT_DEG, q = sh >> 6, r = sh & 63;
    for (int w = 0; w < PW; w++) {
      a[w + q] ^= g_phi[w] << r;
      if (r) a[w + q + 1] ^= g_phi[w] >> (64 - r);
    }
  }
}
static void poly_sqrmod(uint64_t* r, const uint64_t* a) {
  uint64_t t[2 * PW + 2];
  memset(t, 0, sizeof t);
  for (int i = 0; i < MT_DEG; i++) if (pbit(a, i)) pflip(t, 2 * i);
  poly_reduce_fast(t);
  memcpy(r, t, PW * 8);
}
static void poly_mulx(uint64_t* a) {   /* a = a * x mod phi */
  int top = pbit(a, MT_DEG - 1);
  for (int w = PW - 1; w > 0; w--) a[w] = (a[w] << 1) | (a[w - 1] >> 63);
  a[0] <<= 1;
  if (top) {
    pflip(a, MT_DEG);
    for (int w = 0; w < PW; w++) a[w] ^= g_phi[w];
  }
}
/* g = x^N mod phi by left-to-right square-and-multiply */
static int mt_jump_poly(const big* N, uint64_t* g) {
  int rc = mt_need_phi();
  if (rc) return rc;
  memset(g, 0, PW * 8);
  g[0] = 1;
  for (int i = big_nbits(N) - 1; i >= 0; i--) {
    poly_sqrmod(g, g);
    if (big_bit(N, i)) poly_mulx(g);
  }
  return OR_OK;
}
/* g(A) applied to a state at a block boundary (index 624): with seq the raw
   words continued from its window, g(A) Y = sum over the set coefficients i
   of the window starting i words later (equation g_v); the oldest word keeps
   only its top bit (no later output depends on the others). */
static int mt_apply_window(or_mt* st, const uint64_t* g) {
  const int len = MT_DEG - 1 + MT_N;
  uint32_t* seq = (uint32_t*)malloc((size_t)len * 4);
  if (!seq) return OR_ENOMEM;
  for (int j = 0; j < MT_N; j++) seq[j] = st->mt[j];
  for (int j = MT_N; j < len; j++) seq[j] = mt_recur(seq[j - MT_N], seq[j - MT_N + 1], seq[j - MT_N + MT_M]);
  uint32_t res[MT_N];
  memset(res, 0, sizeof res);
  for (int i = 0; i < MT_DEG; i++)
    if (pbit(g, i))
      for (int t = 0; t < MT_N; t++) res[t] ^= seq[i + t];
  memcpy(st->mt, res, sizeof res);
  st->mt[0] &= 0x80000000u;
  st->mti = MT_N;
  free(seq);
  return OR_OK;
}
/* r = a * b mod phi: the carry-less schoolbook product, then reduction */
static void poly_mulmod(uint64_t* r, const uint64_t* a, const uint64_t* b) {
  uint64_t t[2 * PW + 2];
  memset(t, 0, sizeof t);
  for (int i = 0; i < MT_DEG; i++) {
    if (!pbit(a, i)) continue;
    int q = i >> 6, sh = i & 63;
    for (int w = 0; w < PW; w++) {
      t[w + q] ^= b[w] << sh;
      if (sh) t[w + q + 1] ^= b[w] >> (64 - sh);
    }
  }
  poly_reduce_fast(t);
  memcpy(r, t, PW * 8);
}
/* A^N applied to the state; states in the middle of a block first consume
   the rest of the block, so that the polynomial acts on a window of 624
   consecutive raw words whose next output is the tempered successor word.
   The result window is canonical: the low 31 bits of its oldest word, which
   no later output depends on, are cleared. */
static int mt_skip(or_mt* st, const big* Nin) {
  if (st->mti > MT_N) return OR_EINVAL;
  big N = *Nin;
  if (big_is_zero(&N)) return OR_OK;
  uint64_t rest = MT_N - st->mti;
  if (big_le_small(&N, rest)) { st->mti += (uint32_t)N.w[0]; return OR_OK; }
  big_sub_small(&N, rest);
  st->mti = MT_N;
  uint64_t* g = (uint64_t*)malloc(PW * 8);
  if (!g) return OR_ENOMEM;
  int rc = mt_jump_poly(&N, g);
  if (!rc) rc = mt_apply_window(st, g);
  free(g);
  return rc;
}

/* ======================================================================== */
/* GM / GQ torus-map ensembles: x_i^(n) = k x_i^(n-1) - q x_i^(n-2) mod g,   */
/* i = 0..s-1 (paper equation rec1; parameters k, q, g, v of the paper's    */
/* parameter table).                                                         */
/* ======================================================================== */
typedef struct {
  uint64_t k, q, g, p;       /* g = p * 2^t with p prime */
  int v, s;                  /* digit bits per element, ensemble size */
  int steps_per_super, words_per_super;
} gm_par;

#define GM_SMAX 32
typedef struct { uint64_t xp[GM_SMAX]; uint64_t xc[GM_SMAX]; uint32_t off; uint32_t pad; } or_gm;

static const gm_par GM_PARAMS[8] = {
  /* GM19   */ {15, 28, 524287ULL, 524287ULL, 1, 32, 1, 1},
  /* GM29   */ {4, 2, 536870909ULL, 536870909ULL, 1, 32, 1, 1},
  /* GM31   */ {11, 14, 2147483647ULL, 2147483647ULL, 1, 32, 1, 1},
  /* GM55   */ {256, 176, 16ULL * 2251799813685119ULL, 2251799813685119ULL, 4, 8, 1, 1},
  /* GM61   */ {24, 74, 2305843009213693951ULL, 2305843009213693951ULL, 1, 32, 1, 1},
  /* GQ58.1 */ {8, 48, 536870912ULL * 536870909ULL, 536870909ULL, 1, 32, 1, 1},
  /* GQ58.3 */ {8, 48, 536870912ULL * 536870909ULL, 536870909ULL, 3, 12, 8, 9},
  /* GQ58.4 */ {8, 48, 536870912ULL * 536870909ULL, 536870909ULL, 4, 8, 1, 1},
};
static const gm_par* gm_par_of(int gen) { return &GM_PARAMS[gen - OR_GM19]; }

/* one step of one element: returns x^(n+1) from (x^(n), x^(n-1)) */
static uint64_t gm_step_elem(uint64_t k, uint64_t q, uint64_t g, uint64_t xc, uint64_t xp) {
  u128 t = (u128)k * xc + (u128)q * (g - xp);   /* k x - q x' + q g, nonnegative */
  return (uint64_t)(t % g);
}
static uint32_t gm_digit(uint64_t x, int v, uint64_t g) { return (uint32_t)(((u128)x << v) / g); }

/* one ensemble step: advance every element, return the s*v output bits
   (element 0 in the most significant position) */
static uint64_t gm_ensemble_step(const gm_par* P, or_gm* st) {
  uint64_t bits = 0;
  for (int i = 0; i < P->s; i++) {
    uint64_t nx = gm_step_elem(P->k, P->q, P->g, st->xc[i], st->xp[i]);
    st->xp[i] = st->xc[i];
    st->xc[i] = nx;
    bits |= (uint64_t)gm_digit(nx, P->v, P->g) << (P->s * P->v - P->v * (i + 1));
  }
  return bits;
}
/* the words of one super-step (1 step -> 1 word, or 8 steps of 36 bits -> 9
   words); advances st by steps_per_super steps */
static void gm_super(const gm_par* P, or_gm* st, uint32_t* words) {
  int nbits = P->s * P->v;
  int total = nbits * P->steps_per_super;   /* 32 or 288 */
  unsigned char bit[288];
  int pos = 0;
  for (int stp = 0; stp < P->steps_per_super; stp++) {
    uint64_t b = gm_ensemble_step(P, st);
    for (int i = nbits - 1; i >= 0; i--) bit[pos++] = (unsigned char)((b >> i) & 1u);
  }
  for (int w = 0; w < total / 32; w++) {
    uint32_t word = 0;
    for (int i = 0; i < 32; i++) word = (word << 1) | bit[32 * w + i];
    words[w] = word;
  }
}
static void gm_generate_words(int gen, or_gm* st, uint32_t* out, uint64_t n) {
  const gm_par* P = gm_par_of(gen);
  uint32_t buf[9];
  uint64_t i = 0;
  uint32_t off = st->off;
  while (i < n) {
    or_gm next = *st;
    gm_super(P, &next, buf);
    while (off < (uint32_t)P->words_per_super && i < n) out[i++] = buf[off++];
    if (off == (uint32_t)P->words_per_super) {
      *st = next;
      off = 0;
    }
    st->off = off;
  }
}
/* M = ((k, -q), (1, 0)) acting on (x^(n), x^(n-1)) */
typedef struct { uint64_t a, b, c, d; } m2;
static m2 m2_mul(m2 P, m2 Q, uint64_t g) {
  m2 R;
  R.a = (uint64_t)(((u128)P.a * Q.a + (u128)P.b * Q.c) % g);
  R.b = (uint64_t)(((u128)P.a * Q.b + (u128)P.b * Q.d) % g);
  R.c = (uint64_t)(((u128)P.c * Q.a + (u128)P.d * Q.c) % g);
  R.d = (uint64_t)(((u128)P.c * Q.b + (u128)P.d * Q.d) % g);
  return R;
}
static m2 gm_matpow(uint64_t k, uint64_t q, uint64_t g, const big* N) {
  m2 M = {k % g, (g - q % g) % g, 1 % g, 0};
  m2 R = {1 % g, 0, 0, 1 % g};
  int nb = big_nbits(N);
  for (int i = 0; i < nb; i++) {
    if (big_bit(N, i)) R = m2_mul(M, R, g);
    M = m2_mul(M, M, g);
  }
  return R;
}
static void m2_apply(m2 R, uint64_t g, uint64_t* xc, uint64_t* xp) {
  uint64_t nc = (uint64_t)(((u128)R.a * *xc + (u128)R.b * *xp) % g);
  uint64_t np = (uint64_t)(((u128)R.c * *xc + (u128)R.d * *xp) % g);
  *xc = nc; *xp = np;
}
static void gm_skip(int gen, or_gm* st, const big* Nwords) {
  const gm_par* P = gm_par_of(gen);
  big pos = *Nwords;
  big_add_small(&pos, st->off);
  uint64_t rem = big_divmod_small(&pos, (uint64_t)P->words_per_super);  /* pos = super-steps */
  big_mul_small(&pos, (uint64_t)P->steps_per_super);                    /* pos = steps */
  m2 R = gm_matpow(P->k, P->q, P->g, &pos);
  for (int i = 0; i < P->s; i++) m2_apply(R, P->g, &st->xc[i], &st->xp[i]);
  st->off = (uint32_t)rem;
}
static void gm_seed(int gen, or_gm* st, uint64_t seed) {
  const gm_par* P = gm_par_of(gen);
  memset(st, 0, sizeof *st);
  uint64_t sm = seed_start(seed, gen);
  for (int i = 0; i < P->s; i++) {
    do {
      st->xp[i] = draw_below(&sm, P->g);
      st->xc[i] = draw_below(&sm, P->g);
    } while (st->xp[i] % P->p == 0 && st->xc[i] % P->p == 0);
  }
}

/* ======================================================================== */
/* block splitting: stream id = base state jumped ahead id * L outputs,     */
/* L = 2^e outputs (GQ58.3: 2^e ensemble steps = 9 * 2^(e-3) words); e per  */
/* initialising function of the paper's stream table.                        */
/* ======================================================================== */
static const short BLOCK_LOG2[OR_NGEN][5] = {
  /*            DEFAULT SEQ SHORT MEDIUM LONG */
  /* MT19937 */ {-1, 432, -1, -1, -1},
  /* MRG32K3A*/ {-1, 127, -1, -1, -1},
  /* LFSR113 */ {-1, 34, -1, -1, 80},
  /* GM19    */ {-1, 23, -1, -1, -1},
  /* GM29    */ {-1, -1, 27, 33, 40},
  /* GM31    */ {-1, -1, 27, 33, 40},
  /* GM55    */ {-1, -1, 34, -1, 67},
  /* GM61    */ {-1, 34, -1, -1, 85},
  /* GQ58.1  */ {-1, -1, 27, 33, 40},
  /* GQ58.3  */ {-1, -1, 27, 33, 40},
  /* GQ58.4  */ {-1, -1, 27, 33, 40},
};

static int valid_gen(int gen) { return gen >= 0 && gen < OR_NGEN; }

int or_block_log2(int gen, int variant) {
  if (!valid_gen(gen) || variant < 0 || variant > 4) return OR_EINVAL;
  if (variant == OR_VAR_DEFAULT) {
    int e = BLOCK_LOG2[gen][OR_VAR_SEQ];
    return e >= 0 ? e : BLOCK_LOG2[gen][OR_VAR_SHORT];
  }
  int e = BLOCK_LOG2[gen][variant];
  return e >= 0 ? e : OR_EUNSUPPORTED;
}

/* ======================================================================== */
/* exported entry points                                                    */
/* ======================================================================== */
int or_state_bytes(int gen) {
  switch (gen) {
    case OR_MT19937: return (int)sizeof(or_mt);
    case OR_MRG32K3A: return (int)sizeof(or_mrg);
    case OR_LFSR113: return (int)sizeof(or_lfsr);
    default: return valid_gen(gen) ? (int)sizeof(or_gm) : OR_EINVAL;
  }
}

int or_seed(int gen, uint64_t seed, void* st) {
  if (!valid_gen(gen) || !st) return OR_EINVAL;
  memset(st, 0, (size_t)or_state_bytes(gen));
  switch (gen) {
    case OR_MT19937: mt_seed((or_mt*)st, seed); break;
    case OR_MRG32K3A: mrg_seed((or_mrg*)st, seed); break;
    case OR_LFSR113: lfsr_seed((or_lfsr*)st, seed); break;
    default: gm_seed(gen, (or_gm*)st, seed); break;
  }
  return OR_OK;
}

uint64_t or_default_seed(int gen) {
  switch (gen) {
    case OR_MT19937: return 5489;
    case OR_MRG32K3A: return 12345;
    case OR_LFSR113: return 12345;
    default: return 0;
  }
}

int or_init_default(int gen, void* st) {
  if (!valid_gen(gen) || !st) return OR_EINVAL;
  return or_seed(gen, or_default_seed(gen), st);
}

static int skip_big(int gen, void* st, const big* N) {
  switch (gen) {
    case OR_MT19937: return mt_skip((or_mt*)st, N);
    case OR_MRG32K3A: mrg_skip((or_mrg*)st, N); return OR_OK;
    case OR_LFSR113: lfsr_skip((or_lfsr*)st, N); return OR_OK;
    default: gm_skip(gen, (or_gm*)st, N); return OR_OK;
  }
}

int or_skipahead(int gen, void* st, const uint64_t* limbs, int nlimbs) {
  if (!valid_gen(gen) || !st) return OR_EINVAL;
  big N;
  if (big_load(&N, limbs, nlimbs)) return OR_EINVAL;
  return skip_big(gen, st, &N);
}

/* distance id * L in outputs; 0 or an error */
static int stream_distance(int gen, int variant, uint64_t id, big* N) {
  int e = or_block_log2(gen, variant);
  if (e < 0) return e;
  memset(N, 0, sizeof *N);
  N->w[0] = id;
  if (gen == OR_GQ58X3) {
    /* 2^e steps = 2^(e-3) super-steps of 9 words */
    big_mul_small(N, 9);
    e -= 3;
  }
  for (int i = 0; i < e; i++) big_mul_small(N, 2);
  return OR_OK;
}

int or_stream_distance(int gen, int variant, uint64_t id, uint64_t* limbs8) {
  big N;
  int rc = stream_distance(gen, variant, id, &N);
  if (rc) return rc;
  for (int i = 0; i < NLIMB; i++) limbs8[i] = N.w[i];
  return OR_OK;
}

int or_init_stream(int gen, int variant, const void* base, uint64_t id, void* st) {
  if (!valid_gen(gen) || !st) return OR_EINVAL;
  big N;
  int rc = stream_distance(gen, variant, id, &N);
  if (rc) return rc;
  if (base) memcpy(st, base, (size_t)or_state_bytes(gen));
  else or_init_default(gen, st);
  return skip_big(gen, st, &N);
}

int or_generate(int gen, void* st, int dtype, void* out, uint64_t n) {
  if (!valid_gen(gen) || !st || dtype < OR_U32 || dtype > OR_F64) return OR_EINVAL;
  if (n == 0) return OR_OK;
  if (!out) return OR_EINVAL;
  uint32_t* words = (dtype == OR_U32) ? (uint32_t*)out : (uint32_t*)malloc(n * 4);
  if (!words) return OR_ENOMEM;
  switch (gen) {
    case OR_MT19937: for (uint64_t i = 0; i < n; i++) words[i] = mt_next((or_mt*)st); break;
    case OR_MRG32K3A: for (uint64_t i = 0; i < n; i++) words[i] = mrg_next((or_mrg*)st); break;
    case OR_LFSR113: for (uint64_t i = 0; i < n; i++) words[i] = lfsr_next((or_lfsr*)st); break;
    default: gm_generate_words(gen, (or_gm*)st, words, n); break;
  }
  if (dtype == OR_F32) {
    float* f = (float*)out;
    for (uint64_t i = 0; i < n; i++) f[i] = word_to_f32(words[i]);
  } else if (dtype == OR_F64) {
    double* d = (double*)out;
    if (gen == OR_MRG32K3A)
      for (uint64_t i = 0; i < n; i++) d[i] = mrg_to_f64(words[i]);
    else
      for (uint64_t i = 0; i < n; i++) d[i] = word_to_f64(words[i]);
  }
  if (dtype != OR_U32) free(words);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* building blocks exposed for the pins                                     */
/* ------------------------------------------------------------------------ */
int or_mt_charpoly(uint64_t* out /* PW words, x^19937 omitted */) {
  int rc = mt_need_phi();
  if (rc) return rc;
  memcpy(out, g_phi, sizeof g_phi);
  return MT_DEG;
}
int or_mt_jump_poly(const uint64_t* limbs, int nlimbs, uint64_t* out /* PW words */) {
  big N;
  if (big_load(&N, limbs, nlimbs)) return OR_EINVAL;
  return mt_jump_poly(&N, out);
}
/* the bit-level reduction, for a pin that checks the word-level one */
int or_mt_reduce_bitwise(uint64_t* a /* 2*PW+2 words */) {
  int rc = mt_need_phi();
  if (rc) return rc;
  poly_reduce(a);
  return OR_OK;
}
int or_mt_reduce_words(uint64_t* a /* 2*PW+2 words */) {
  int rc = mt_need_phi();
  if (rc) return rc;
  poly_reduce_fast(a);
  return OR_OK;
}
/* 3x3 matrix power mod m (entries < m < 2^63) */
int or_mat3_pow(const uint64_t* M9, uint64_t m, const uint64_t* limbs, int nlimbs, uint64_t* out9) {
  big N;
  if (m < 2 || big_load(&N, limbs, nlimbs)) return OR_EINVAL;
  m3 A;
  for (int i = 0; i < 9; i++) A.a[i / 3][i % 3] = M9[i] % m;
  m3 R = m3_pow(&A, &N, m);
  for (int i = 0; i < 9; i++) out9[i] = R.a[i / 3][i % 3];
  return OR_OK;
}
/* GM recurrence with arbitrary (k, q, g): one step and a jump of N steps,
   on (x^(n), x^(n-1)) = (*xc, *xp) */
int or_gm_generic_step(uint64_t k, uint64_t q, uint64_t g, uint64_t* xc, uint64_t* xp) {
  if (g < 2 || *xc >= g || *xp >= g) return OR_EINVAL;
  uint64_t nx = gm_step_elem(k % g, q % g, g, *xc, *xp);
  *xp = *xc; *xc = nx;
  return OR_OK;
}
int or_gm_generic_jump(uint64_t k, uint64_t q, uint64_t g, const uint64_t* limbs, int nlimbs,
                       uint64_t* xc, uint64_t* xp) {
  big N;
  if (g < 2 || *xc >= g || *xp >= g || big_load(&N, limbs, nlimbs)) return OR_EINVAL;
  m2 R = gm_matpow(k, q, g, &N);
  m2_apply(R, g, xc, xp);
  return OR_OK;
}
/* LFSR component with arbitrary (p, q, s): one step and a jump of N steps */
uint32_t or_lfsr_comp_step(uint32_t z, int p, int q, int s) { return lfsr_comp_step(z, p, q, s); }
uint32_t or_lfsr_comp_jump(uint32_t z, int p, int q, int s, const uint64_t* limbs, int nlimbs) {
  big N;
  if (big_load(&N, limbs, nlimbs)) return 0;
  return lfsr_comp_jump(z, p, q, s, &N);
}
/* a * b mod phi (reduced inputs: degree < 19937) */
int or_mt_poly_mulmod(const uint64_t* a, const uint64_t* b, uint64_t* out /* PW words each */) {
  int rc = mt_need_phi();
  if (rc) return rc;
  poly_mulmod(out, a, b);
  return OR_OK;
}
/* g(A) applied to an MT19937 state at a block boundary (index 624) */
int or_mt_apply_poly(void* st, const uint64_t* g /* PW words, reduced */) {
  or_mt* m = (or_mt*)st;
  if (m->mti != MT_N) return OR_EINVAL;
  return mt_apply_window(m, g);
}
/* x^(2^n) mod phi by n squarings (for an irreducibility pin) */
int or_mt_frobenius(int n, uint64_t* out /* PW words */) {
  int rc = mt_need_phi();
  if (rc) return rc;
  if (n < 0) return OR_EINVAL;
  memset(out, 0, PW * 8);
  out[0] = 2;   /* x */
  for (int i = 0; i < n; i++) poly_sqrmod(out, out);
  return OR_OK;
}
