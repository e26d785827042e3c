// prand_generate_noalloc: the sectioned fill of prand_generate with its
// scratch (section start states, their distances, the copied-in state) in a
// file-scope device array instead of memory allocated per call.
//
// The array's name is a host-side stand-in in host code: its device address
// is looked up once per device (hipGetSymbolAddress, from the context set-up
// with the device current) and only that address is used afterwards.
#include <hip/hip_runtime.h>

#include <mutex>

#include "prand_impl.h"

namespace {

constexpr size_t kNoAllocBytes = PRAND_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_setup_mu;               // guards g_scratch
void* g_scratch[kMaxDevices] = {};   // device address of `scratch` per device
std::mutex g_call_mu[kMaxDevices];   // one call at a time per device's array

}  // namespace

hipError_t prand::noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_setup_mu);
  if (g_scratch[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch[device] = p;
  return hipSuccess;
}

extern "C" int prand_generate_noalloc(prand_ctx* c, int gen, void* h_state, int dtype, void* d_out, uint64_t n,
                                      void* stream) {
  if (!c || gen < 0 || gen >= PRAND_NUM_GENERATORS || dtype < PRAND_U32 || dtype > PRAND_F64 || !h_state)
    return PRAND_EINVAL;
  if (n == 0) return PRAND_OK;
  if (!d_out) return PRAND_EINVAL;
  if (n > (1ull << 40)) return PRAND_ERANGE;
  if (c->device < 0 || c->device >= kMaxDevices) return PRAND_EINVAL;
  void* p;
  {
    std::lock_guard<std::mutex> lk(g_setup_mu);
    p = g_scratch[c->device];
  }
  if (!p) return PRAND_ENOTREADY;
  if (gen == PRAND_MT19937 && !prand::mt_tables_ready(c)) return PRAND_ENOTREADY;
  prand::DeviceGuard g(c->device);
  std::lock_guard<std::mutex> lk(g_call_mu[c->device]);
  return prand::generate_host_state(c, gen, h_state, dtype, d_out, n, (hipStream_t)stream, p, kNoAllocBytes);
}
