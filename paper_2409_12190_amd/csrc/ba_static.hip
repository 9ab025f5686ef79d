// Device scratch of the allocation-free binding (ba_problem_bind_static): one
// file-scope array, present on every GPU the library runs on, of a fixed
// size.  Host code never uses the array's name as an address: the device
// address of each GPU's copy is resolved once per device with
// hipGetSymbolAddress and cached here.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ba_internal.h"

namespace ba {

namespace {

__device__ __align__(256) char scratch[STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};

}  // namespace

hipError_t static_scratch(int device, void** ptr) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  int current = -1;
  hipError_t e = hipGetDevice(&current);
  if (e != hipSuccess) return e;
  if (current != device) return hipErrorInvalidDevice;  // resolve with the device current
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[device] = p;
  }
  *ptr = g_ptr[device];
  return hipSuccess;
}

}  // namespace ba
