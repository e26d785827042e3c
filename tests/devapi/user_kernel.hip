// Test-side user kernels built on include/prand_device.h: one state per
// thread, drawn with the header's device functions exactly as an
// application kernel would; and the same loop on the host (the header's
// functions compile for the CPU too).  Not part of the library.
#include <hip/hip_runtime.h>

#include "prand_device.h"

namespace {

// out[t * n + i] = i-th value drawn from state t (advanced in place)
template <int DT>
__global__ void draw_kernel(int gen, char* states, size_t sb, uint32_t count, uint64_t n, void* out) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  void* st = states + (size_t)t * sb;
  for (uint64_t i = 0; i < n; i++) {
    const uint64_t o = (uint64_t)t * n + i;
    if (DT == PRAND_U32) ((uint32_t*)out)[o] = prand_next(gen, st);
    else if (DT == PRAND_F32) ((float*)out)[o] = prand_uniform_float(gen, st);
    else ((double*)out)[o] = prand_uniform_double(gen, st);
  }
}

// sums[t] = left-to-right double sum of n uniform doubles drawn from state
// t: the numbers are consumed in registers, only the sum is stored
__global__ void sum_kernel(int gen, char* states, size_t sb, uint32_t count, uint64_t n, double* sums) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  void* st = states + (size_t)t * sb;
  double acc = 0.0;
  for (uint64_t i = 0; i < n; i++) acc += prand_uniform_double(gen, st);
  sums[t] = acc;
}

size_t blob_bytes(int gen) {
  switch (gen) {
    case PRAND_MT19937: return sizeof(prand_mt19937_state);
    case PRAND_MRG32K3A: return sizeof(prand_mrg32k3a_state);
    case PRAND_LFSR113: return sizeof(prand_lfsr113_state);
    default: return sizeof(prand_gm_state);
  }
}

}  // namespace

extern "C" size_t devapi_state_bytes(int gen) { return blob_bytes(gen); }

extern "C" int devapi_draw(int gen, int dtype, void* d_states, uint32_t count, uint64_t n, void* d_out,
                           void* stream) {
  if (gen < 0 || gen >= PRAND_NUM_GENERATORS || count == 0) return -1;
  const dim3 grid((count + 63) / 64), block(64);
  const size_t sb = blob_bytes(gen);
  hipStream_t st = (hipStream_t)stream;
  if (dtype == PRAND_U32)
    hipLaunchKernelGGL(draw_kernel<PRAND_U32>, grid, block, 0, st, gen, (char*)d_states, sb, count, n, d_out);
  else if (dtype == PRAND_F32)
    hipLaunchKernelGGL(draw_kernel<PRAND_F32>, grid, block, 0, st, gen, (char*)d_states, sb, count, n, d_out);
  else
    hipLaunchKernelGGL(draw_kernel<PRAND_F64>, grid, block, 0, st, gen, (char*)d_states, sb, count, n, d_out);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

extern "C" int devapi_sum(int gen, void* d_states, uint32_t count, uint64_t n, double* d_sums, void* stream) {
  if (gen < 0 || gen >= PRAND_NUM_GENERATORS || count == 0) return -1;
  hipLaunchKernelGGL(sum_kernel, dim3((count + 63) / 64), dim3(64), 0, (hipStream_t)stream, gen, (char*)d_states,
                     blob_bytes(gen), count, n, d_sums);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

// the draw loop of draw_kernel on the CPU, over host states
extern "C" int hostapi_draw(int gen, int dtype, void* h_states, uint32_t count, uint64_t n, void* h_out) {
  if (gen < 0 || gen >= PRAND_NUM_GENERATORS) return -1;
  const size_t sb = blob_bytes(gen);
  for (uint32_t t = 0; t < count; t++) {
    void* st = (char*)h_states + (size_t)t * sb;
    for (uint64_t i = 0; i < n; i++) {
      const uint64_t o = (uint64_t)t * n + i;
      if (dtype == PRAND_U32) ((uint32_t*)h_out)[o] = prand_next(gen, st);
      else if (dtype == PRAND_F32) ((float*)h_out)[o] = prand_uniform_float(gen, st);
      else ((double*)h_out)[o] = prand_uniform_double(gen, st);
    }
  }
  return 0;
}
