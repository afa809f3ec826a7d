// Small host-side helpers of the library.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/ckks_lt.h"

namespace ckks {

int params_create(const ckks_params_desc* d, ckks_params** out);
void params_destroy(ckks_params* P);
uint32_t galois(const ckks_params* P, long r);

// Owns a freshly created object until release(); destroys it otherwise.
template <class T>
struct Cleanup {
  T* p;
  explicit Cleanup(T* x) : p(x) {}
  ~Cleanup() {
    if (p) params_destroy(p);
  }
  T* release() {
    T* x = p;
    p = nullptr;
    return x;
  }
};

// Bump allocator over the caller's workspace.  With base == nullptr it only
// measures (the same code path sizes and then runs a call).
struct Workspace {
  uint8_t* base = nullptr;
  size_t off = 0, peak = 0;
  size_t limb_bytes = 0;
  uint64_t* limbs(size_t count) {
    const size_t bytes = (count * limb_bytes + 255) & ~(size_t)255;
    uint64_t* p = base ? reinterpret_cast<uint64_t*>(base + off) : nullptr;
    off += bytes;
    peak = std::max(peak, off);
    return p;
  }
  size_t mark() const { return off; }
  void reset(size_t m) { off = m; }
};

}  // namespace ckks
