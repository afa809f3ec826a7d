// Device scratch of the no-allocation LT entry point (ckks_lt_eval_noalloc).
//
// One file-scope device array per GPU, made when the code object is loaded on
// that GPU and held until the process ends.  Host code never uses the array's
// name as an address (on the host it is only a stand-in for the symbol): the
// device address is looked up once per device, with that device current, and
// kept; every later use goes through that pointer.
#include <mutex>

#include "internal.hpp"

namespace ckks {

namespace {

constexpr int kMaxDevices = 64;

__device__ __align__(256) uint8_t scratch[CKKS_LT_NOALLOC_MAX_WS];

std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {};

}  // namespace

int scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices || !out) return CKKS_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_ptr[device]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != device) return CKKS_E_DEVICE;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return CKKS_E_DEVICE;
    }
    scratch_ptr[device] = p;
  }
  *out = scratch_ptr[device];
  return CKKS_OK;
}

}  // namespace ckks
