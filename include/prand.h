/*
 * prand.h -- C ABI of an MI355X (gfx950) library for bulk parallel uniform
 * pseudorandom number generation with the eleven generators of Barash &
 * Shchur, "PRAND: GPU accelerated parallel random number generation library",
 * Comput. Phys. Commun. 185 (2014) 1343.
 *
 * Conventions shared by every entry point
 *  - Every function returns int: PRAND_OK (0) on success, a negative
 *    PRAND_E* code on failure; prand_strerror() names a code.  No C++
 *    exception crosses this boundary.  On failure nothing has been enqueued
 *    and no state has been modified, except PRAND_EHIP, which reports a HIP
 *    runtime error (prand_last_hip_error() gives the hipError_t value).
 *  - "h_" pointers are host memory, "d_" pointers are device memory of the
 *    context's device.  The caller owns every state and output buffer; the
 *    context owns only its constant tables.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Functions taking
 *    only device buffers are asynchronous: they enqueue kernels on `stream`
 *    and return.  Functions taking a host state block until the state has
 *    been updated (the paper's host interface, section "Function call
 *    interface").
 *  - A generator state is a plain-old-data blob of prand_state_bytes(gen)
 *    bytes, little-endian, with the same layout on host and device, so it can
 *    be copied between them freely (paper, section "Function call
 *    interface": states may be advanced on the CPU and continued on the GPU):
 *      MT19937   uint32 mt[624], uint32 index (0..624), uint32 pad[3]
 *      MRG32K3A  uint32 x_n, x_{n-1}, x_{n-2} (mod m1), y_n, y_{n-1}, y_{n-2} (mod m2)
 *      LFSR113   uint32 z[4]
 *      GM/GQ     uint64 xprev[32], uint64 xcur[32] (elements >= s are 0),
 *                uint32 word offset inside the current 8-step block (GQ58.3
 *                only, else 0), uint32 pad
 *  - Outputs: word i of a stream is the i-th 32-bit output; PRAND_F32 stores
 *    (w >> 8) * 2^-24, PRAND_F64 stores w * 2^-32, except MRG32K3A whose
 *    PRAND_F64 stores z * RN(1/(m1+1)) in (0,1) (the generator's usual
 *    normalisation).  Many-stream outputs are row-major: out[stream][i].
 *  - Distances ("skip ahead", block lengths) count 32-bit outputs, given as
 *    little-endian uint64 limbs; up to 8 limbs (2^512).
 */
#ifndef PRAND_H
#define PRAND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The generators of the paper's Table 2 ("Parameters of the generators"). */
enum prand_gen {
  PRAND_MT19937 = 0,   /* Matsumoto-Nishimura Mersenne twister, period 2^19937-1 */
  PRAND_MRG32K3A = 1,  /* L'Ecuyer's combined MRG, matrices A, B of the MRG32K3A jump section */
  PRAND_LFSR113 = 2,   /* four combined shift registers, relations lfsrRel1/lfsrOutput */
  PRAND_GM19 = 3,      /* torus-map ensembles, recurrence rec1 with (k, q, g, v) of Table 2 */
  PRAND_GM29 = 4,
  PRAND_GM31 = 5,
  PRAND_GM55 = 6,
  PRAND_GM61 = 7,
  PRAND_GQ58X1 = 8,
  PRAND_GQ58X3 = 9,    /* 36 output bits per step: 9 words per 8 steps */
  PRAND_GQ58X4 = 10
};
#define PRAND_NUM_GENERATORS 11

enum prand_dtype { PRAND_U32 = 0, PRAND_F32 = 1, PRAND_F64 = 2 };

/* Stream-initialising functions of the paper's Table 4 ("Initialization of
   pseudorandom streams"): rng_init_sequence_, rng_init_short_sequence_,
   rng_init_medium_sequence_, rng_init_long_sequence_.  PRAND_SEQ_DEFAULT is
   PRAND_SEQ where the generator has it, else PRAND_SEQ_SHORT. */
enum prand_variant {
  PRAND_SEQ_DEFAULT = 0,
  PRAND_SEQ = 1,
  PRAND_SEQ_SHORT = 2,
  PRAND_SEQ_MEDIUM = 3,
  PRAND_SEQ_LONG = 4
};

#define PRAND_OK 0
#define PRAND_EINVAL (-1)        /* null pointer, bad enum value, limb count out of range */
#define PRAND_EUNSUPPORTED (-2)  /* variant not listed in Table 4 for this generator */
#define PRAND_ERANGE (-3)        /* size beyond what the entry point accepts */
#define PRAND_EHIP (-4)          /* HIP runtime error, see prand_last_hip_error() */
#define PRAND_ENOMEM (-5)        /* allocation failed */
#define PRAND_ENODEV (-6)        /* no usable gfx950 device */
#define PRAND_EBUSY (-7)         /* serving queue full: request rejected */
#define PRAND_ENOTREADY (-8)     /* context tables the call needs are not built, and it may not build them */

typedef struct prand_ctx prand_ctx;

/* Text for an error code.  Never NULL; the string is static. */
const char* prand_strerror(int code);

/* hipError_t of the most recent PRAND_EHIP returned through this context. */
int prand_last_hip_error(const prand_ctx* ctx);

/* Create a context on HIP device `hip_device`: uploads the jump-ahead tables
   (the counterpart of the paper's rng_init_device_consts_, section "Function
   call interface for MRG32K3A / MT19937"): matrix powers A^(2^j), B^(2^j) for
   MRG32K3A, 32x32 F2 matrix powers for LFSR113, 2x2 matrix powers for GM/GQ,
   and x^(2^j) mod phi for MT19937 (equation g_v; phi is computed once by
   Berlekamp-Massey).  The MT19937 tables (656 MB: the ladder, the digit
   tables of block splitting and the 65536 precomputed top-16-bit states)
   are built when a call first needs them and are shared by all contexts on
   the same device, freed with the last of them.  *ctx is set to NULL on
   failure. */
int prand_ctx_create(prand_ctx** ctx, int hip_device);

/* Free the context's device tables (rng_free_device_consts_).  NULL is OK. */
int prand_ctx_destroy(prand_ctx* ctx);

/* Size in bytes of the state blob of `gen` (the paper's rng_state, section
   "Function call interface": one structure per generator holding all of its
   internal state, copied between host and device memory as is); 0 for an
   invalid generator. */
size_t prand_state_bytes(int gen);

/* Block-splitting block length: stream `id` starts id * L outputs into the
   base sequence, L = 2^e ensemble steps (= 2^e outputs except GQ58.3, where
   it is 9 * 2^(e-3) outputs).  Returns e >= 0, or PRAND_EUNSUPPORTED /
   PRAND_EINVAL.  (Paper, section "Parallel streams", Table 4.) */
int prand_block_log2(int gen, int variant);

/* Table 4 metadata: the number of independent sequences and the maximal
   length the paper guarantees for this initialising function. */
int prand_independence_limit(int gen, int variant, double* max_streams, double* max_length);

/* Default state (rng_init_): MT19937 init_genrand(5489), MRG32K3A and
   LFSR113 all words 12345, GM/GQ the seed-0 expansion.  Blocks. */
int prand_init_default(prand_ctx* ctx, int gen, void* h_state);

/* Seeded state.  MT19937: init_genrand(seed) for seed < 2^32, else
   init_by_array over the two 32-bit halves.  MRG32K3A: all six words = seed
   when 1 <= seed < m2.  LFSR113: all four words = seed when
   128 <= seed < 2^32.  Otherwise (and for GM/GQ, per element) SplitMix64
   draws reduced by rejection, from a start state that is the first SplitMix64
   output of seed ^ (0x9E3779B97F4A7C15 * (gen + 1)).  Blocks. */
int prand_seed(prand_ctx* ctx, int gen, uint64_t seed, void* h_state);

/* Host-only forms of prand_seed and prand_init_default (section
   "Function call interface", "Initialization": rng_init_ and its seeded
   form are callable from host code): the same states, computed on the CPU
   by the library's seeding code, with no context and no GPU.  h_state:
   prand_state_bytes(gen) bytes, written.  PRAND_EINVAL for an unknown
   generator or a null state. */
int prand_seed_host(int gen, uint64_t seed, void* h_state);
int prand_init_default_host(int gen, void* h_state);

/* count states from count seeds, on the device: the seeded form of
   rng_init_, which the paper provides in device code too (section
   "Function call interface", "Initialization").  d_seeds: count uint64;
   d_states: count state blobs, written.  Asynchronous on `stream`. */
int prand_seed_dev(prand_ctx* ctx, int gen, const uint64_t* d_seeds, uint32_t count,
                   void* d_states, void* stream);

/* Jump a host state ahead by `dist` outputs (rng_skipahead_, section
   "Jumping ahead").  dist: nlimbs little-endian uint64 limbs, 0 <= nlimbs
   <= 8.  Runs on the device; blocks. */
int prand_skipahead(prand_ctx* ctx, int gen, void* h_state, const uint64_t* h_dist, int nlimbs);

/* Jump count device states ahead (rng_skipahead_ in device code, section
   "Function call interface", "Jumping ahead"; the jump methods of section
   "Parallel streams of pseudorandom numbers").  d_dist holds nlimbs limbs per
   stream (count * nlimbs uint64, stream-major) when per_stream != 0, else one
   distance of nlimbs limbs shared by all streams; 0 <= nlimbs <= 8.  States
   are updated in place.  Asynchronous on `stream`. */
int prand_skipahead_dev(prand_ctx* ctx, int gen, void* d_states, uint32_t count,
                        const uint64_t* d_dist, int nlimbs, int per_stream, void* stream);

/* Stream `id` by block splitting (rng_init_sequence_ and variants): the
   default state jumped ahead id * L outputs.  Any uint64 id is accepted;
   independence is only claimed below prand_independence_limit().  Blocks. */
int prand_init_stream(prand_ctx* ctx, int gen, int variant, uint64_t id, void* h_state);

/* count streams on the device: d_states[i] = base jumped id[i] * L.
   d_base_state: a device state blob, or NULL for the default state. */
int prand_init_streams_dev(prand_ctx* ctx, int gen, int variant, const void* d_base_state,
                           const uint64_t* d_ids, uint32_t count, void* d_states, void* stream);

/* Fill d_out with the next n outputs of one host state (rng_generate_gpu_
   array_[float_|double_], section "Multi-threaded generation"): the array is
   cut into sections that jump to their start and fill in parallel; the
   result equals sequential generation for every n (no divisibility or
   power-of-two condition).  h_state is advanced by n.  The section states
   live in a device buffer the context keeps between calls (allocated, or
   grown, only when a call needs more than any earlier one; freed with the
   context); calls on one context are serialised.  Blocks. */
int prand_generate(prand_ctx* ctx, int gen, void* h_state, int dtype, void* d_out, uint64_t n,
                   void* stream);

/* Fill the host array h_out with the next n outputs of one host state
   (rng_generate_array_, section "Multi-threaded generation of pseudorandom
   numbers with GPGPU"): the values are generated on the device exactly as
   by prand_generate, in chunks of up to 2^26 values through one device
   buffer allocated for the call, and copied to the host; h_state is
   advanced by n.  Any n is accepted (the paper's version pads n to a
   multiple of its section count on the device; here the sections need no
   padding).  PRAND_ERANGE when n > 2^40.  Blocks. */
int prand_generate_array(prand_ctx* ctx, int gen, void* h_state, int dtype, void* h_out, uint64_t n);

/* Many independent streams (section "Multi-threaded generation of
   pseudorandom numbers with GPGPU" applied to one state per stream, as in
   the paper's use of block splitting to give every thread block its own
   stream): d_out[s * n_per_stream + i] = output i of stream s, for s < count;
   each d_states[s] is advanced by n_per_stream in place.  PRAND_ERANGE when
   n_per_stream > 2^40 or the output exceeds 2^50 bytes.  Asynchronous on
   `stream`, except that the first MRG32K3A or LFSR113 call with a given
   section length (a function of count and n_per_stream) builds that length's
   section-start table (up to 32 KB of device memory, kept until the context
   is destroyed; a blocking copy), unless `stream` is being captured into a
   graph: calls under capture, and calls past 64 such lengths per generator,
   jump every section through the ladder instead (same outputs, more work). */
int prand_generate_streams(prand_ctx* ctx, int gen, void* d_states, uint32_t count,
                           uint64_t n_per_stream, int dtype, void* d_out, void* stream);

/* prand_generate for callers that cannot allocate device memory (harnesses
   that forbid hipMalloc, tight serving loops): the same arguments, result
   and blocking behaviour, but the section start states, their distances and
   the copied-in state live in a static device array of 4 MiB per GPU
   (PRAND_NOALLOC_SCRATCH_BYTES) instead of memory allocated per call, and no
   hipMalloc, hipFree or allocating library routine is called.  The array is
   reserved by the library on each device where a context is created and is
   held until the process ends.  The section plan is limited to what fits in
   it (at most 1663 MT19937, 7941 GM/GQ, 131048 MRG32K3A and 174730 LFSR113
   sections); the output never depends on the plan.  PRAND_ERANGE when
   n > 2^40.  MT19937 needs the context's jump tables: PRAND_ENOTREADY when no
   earlier MT19937 call on this context (for example prand_init_stream) has
   built them.  Every call on one GPU shares that GPU's array and keeps the
   last call's contents there: the library serialises the calls of one
   process on a device (each call holds the array until its copy-back has
   finished), and calls that overlap from another thread block until then. */
#define PRAND_NOALLOC_SCRATCH_BYTES (4u << 20)
int prand_generate_noalloc(prand_ctx* ctx, int gen, void* h_state, int dtype, void* d_out, uint64_t n,
                           void* stream);

/* ------------------------------------------------------------------------
 * Batched launch: many streams of uneven lengths and mixed generators and
 * dtypes in one launch, replayed from a HIP graph.  Each task is cut into
 * sections that jump to their first output (the sectioning of "Multi-threaded
 * generation"), grouped into per-wavefront tiles; a first kernel computes
 * every section's start state, then three persistent kernels, one per
 * register class (the lane-per-section GM55/GQ58.3/GQ58.4 tiles;
 * MRG32K3A/LFSR113; MT19937 with the v = 1 GM/GQ ensembles), work through
 * their tile lists longest first, every wavefront taking the next tile from
 * its class's device counter -- one after another, each with as many
 * wavefronts as the chip holds, or side by side, each with a share of the
 * chip sized by its work, or the MRG32K3A/LFSR113 class first and then the
 * other two side by side (prand_batch_config.overlap).
 * ------------------------------------------------------------------------ */
typedef struct prand_task {
  int32_t gen;           /* enum prand_gen */
  int32_t dtype;         /* enum prand_dtype */
  uint64_t n;            /* outputs */
  const void* state_in;  /* device state blob (read only) */
  void* state_out;       /* device state blob: state_in advanced by n.  No state_out may
                            overlap any task's state_in; state_out blobs are distinct. */
  void* out;             /* device array of n values of dtype (may be NULL when n = 0) */
} prand_task;

typedef struct prand_batch_config {
  uint32_t waves_per_block; /* wavefronts per workgroup: 1, 2 or 4 (0: 4) */
  uint32_t reg_section;    /* MRG32K3A/LFSR113 outputs per lane section, multiple of 32 (0: 2048) */
  uint32_t gm_section;     /* GM/GQ outputs per element-group section (0: 4096) */
  uint32_t use_graph;      /* 1: capture the launch in a HIP graph and replay it */
  uint32_t lds_chunk_words; /* LDS staging of MRG32K3A/LFSR113 lanes, 16 or 32 words (0: 32):
                               5 or 9 KB per wavefront of their kernel */
  uint32_t overlap;        /* 0: the three class kernels run one after another; 1: side by side,
                              each class's share of the chip sized by its work; 2: the
                              MRG32K3A/LFSR113 class first with the whole chip, then the other
                              two side by side */
} prand_batch_config;

typedef struct prand_batch prand_batch;

/* Plan a batch (tasks are read on the host; the device pointers they hold
   must stay valid while the batch is launched).  cfg NULL: defaults.  The
   batch owns a device scratch area for the section start states (about 1.5 KB
   per tile).  MT19937 tasks longer than 2^24 outputs are run as sections of
   624 * 2^10 outputs, whose start states come from whole-block jumps of the
   task state; a batch with such a task makes the context build its MT19937
   jump tables first, if no earlier call has (a few seconds, once). */
int prand_batch_create(prand_ctx* ctx, const prand_task* h_tasks, uint32_t ntasks, const prand_batch_config* cfg,
                       prand_batch** batch);
/* Enqueue the batch on `stream` (a hipStream_t, NULL = default stream), as
   one graph launch when use_graph is set, else as its kernels.  Launches of
   the same batch must not overlap each other (they share the batch's tile
   counters and scratch). */
int prand_batch_launch(prand_batch* batch, void* stream);
/* Number of tiles (wavefront work items) the plan holds. */
int prand_batch_tiles(const prand_batch* batch, uint32_t* ntiles);
int prand_batch_destroy(prand_batch* batch);

/* Time candidate configurations on these tasks (their outputs and output
   states are overwritten) and return the fastest in *best: each candidate
   scored by the slowest of three launches, then the best three re-timed over
   six launches each and ranked by their mean.  When the
   environment variable PRAND_TUNE_CACHE names a file, results are kept there
   keyed by the device and a signature of the task mix, and reused.  Blocks. */
int prand_batch_autotune(prand_ctx* ctx, const prand_task* h_tasks, uint32_t ntasks, prand_batch_config* best);


/* ------------------------------------------------------------------------
 * Serving loop: a native request loop over one device.  Requests (generator,
 * stream id, length, dtype) arrive at any time from any thread; a worker
 * thread admits them while their output and state fit in a fixed HBM budget,
 * initialises each request's stream by block splitting on a second HIP
 * stream, and runs continuous batching: every loop iteration is one batched
 * launch holding the next chunk of every admitted request, so
 * short requests finish while long ones are still running.  States stay on
 * the device between iterations; outputs stay on the device until released.
 * A request's output equals prand_init_stream(id) followed by generation of n
 * outputs, whatever else is being served.
 * ------------------------------------------------------------------------ */
typedef struct prand_server prand_server;

typedef struct prand_server_config {
  uint64_t hbm_budget;      /* bytes of device memory for outputs and states (0: 16 GiB);
                               reserved by prand_server_create */
  uint64_t iter_numbers;    /* outputs per loop iteration over all requests (0: 2^28) */
  uint64_t min_chunk;       /* smallest per-request share of an iteration (0: 2^16) */
  uint64_t mt_chunk;        /* largest MT19937 chunk per iteration (one wavefront each; 0: 2^20) */
  uint64_t mt_section;      /* MT19937 requests longer than this are cut into up to 256 sections of
                               624 * 2^k outputs (k >= 10) that start from jumped states and run in
                               parallel (0: 2^20) */
  uint32_t max_active;      /* requests generating at once (0: 8192) */
  uint32_t max_queue;       /* waiting requests beyond which submissions are rejected (0: 2^20) */
  uint32_t waves_per_block; /* batch kernel shape, as prand_batch_config (0: defaults) */
  uint32_t reg_section;
  uint32_t gm_section;
  uint32_t pad;
} prand_server_config;

typedef struct prand_request {
  int32_t gen;              /* enum prand_gen */
  int32_t variant;          /* enum prand_variant (stream initialisation) */
  int32_t dtype;            /* enum prand_dtype */
  int32_t pad;
  uint64_t stream_id;       /* block-splitting stream number */
  uint64_t n;               /* outputs, 1 <= n <= 2^40 */
  uint64_t tag;             /* caller's value, returned in the completion */
} prand_request;

typedef struct prand_completion {
  uint64_t ticket;
  uint64_t tag;
  uint64_t n;
  int32_t gen;
  int32_t dtype;
  void* out;                /* device array of n values; valid until prand_server_release(ticket) */
  void* state;              /* device state blob: the stream advanced by n; same lifetime */
  double t_submit;          /* seconds on the server clock (prand_server_clock) */
  double t_admit;           /* memory reserved, initialisation enqueued */
  double t_done;            /* the worker saw the last chunk's launch complete */
} prand_completion;

typedef struct prand_server_stats {
  uint64_t submitted, admitted, rejected, completed, released;
  uint64_t numbers;         /* outputs of completed requests */
  uint64_t iterations;      /* batched launches */
  uint64_t hbm_budget, hbm_used, hbm_peak;
  uint32_t waiting, active; /* requests waiting for memory / admitted and not complete */
  double gpu_busy_s;        /* summed duration of the batched launches */
} prand_server_stats;

/* Start a server on the context's device (cfg NULL: defaults).  Blocks until
   the budget is reserved and the worker runs. */
int prand_server_create(prand_ctx* ctx, const prand_server_config* cfg, prand_server** server);
/* Queue a request.  PRAND_EINVAL for a bad field, PRAND_EUNSUPPORTED for a
   variant the generator lacks, PRAND_ERANGE when its output and state could
   never fit the budget, PRAND_EBUSY when the queue is full; otherwise
   *ticket identifies it.  Thread-safe, does not block on the device. */
int prand_server_submit(prand_server* server, const prand_request* req, uint64_t* ticket);
/* Move up to max completions into out[], oldest first; waits up to wait_ms
   milliseconds for the first one (0: no wait). */
int prand_server_poll(prand_server* server, prand_completion* out, uint32_t max, uint32_t* count, int wait_ms);
/* Give back a completed request's output and state memory. */
int prand_server_release(prand_server* server, uint64_t ticket);
int prand_server_get_stats(prand_server* server, prand_server_stats* stats);
/* Seconds since the server started (the clock of the completion times). */
double prand_server_clock(const prand_server* server);
/* Stop the worker after the admitted requests have finished and free
   everything, including unreleased outputs. */
int prand_server_destroy(prand_server* server);

/* ---- CPU SIMD generation (section "Generation with SSE") ----------------
   Host-only functions, no context and no GPU: the paper's
   rng_get_sse_state_ / rng_sse_generate_.  A SIMD state continues a plain
   state blob of any generator on the CPU with vector instructions (x86-64
   AVX2 and FMA, checked at run time; without them, or when the environment
   variable PRAND_SIMD_DISABLE is set to a non-zero value as the state is
   made, the same state runs plain scalar code).  It holds a buffer of the
   next outputs: MT19937 one 624-word block, LFSR113 eight lanes and
   MRG32K3A four lanes of 512 consecutive outputs each (the lanes are the
   stream cut into runs that start from jumps, so the outputs are in
   sequence order), GM/GQ 1024 ensemble steps (GQ58.3: 128 blocks of 9
   words).  The outputs are exactly those of the plain state.  The blob is
   caller-allocated, prand_simd_state_bytes() bytes, any alignment; it may
   be copied.  A state must not be used by two threads at once. */
size_t prand_simd_state_bytes(void);
/* rng_get_sse_state_: make *simd_state continue the plain state blob h_state
   of generator gen (h_state is read, not changed).  PRAND_EINVAL for a bad
   generator or a null pointer. */
int prand_get_simd_state(int gen, const void* h_state, void* simd_state);
/* rng_sse_generate_: the next 32-bit output (0 for a blob that is not a
   SIMD state). */
uint32_t prand_simd_next(void* simd_state);
/* The next n outputs into h_out as dtype (u32, f32 or f64, the maps of the
   device calls); PRAND_EINVAL for a bad state, dtype or null h_out. */
int prand_simd_fill(void* simd_state, int dtype, void* h_out, uint64_t n);
/* 1 when the state runs the vector code, 0 the scalar code, PRAND_EINVAL
   for a blob that is not a SIMD state. */
int prand_simd_vectorized(const void* simd_state);

#ifdef __cplusplus
}
#endif

#endif /* PRAND_H */
