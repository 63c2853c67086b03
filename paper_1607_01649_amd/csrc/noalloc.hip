// rsvd_factor_noalloc: the fixed-rank factorisation of rsvd_factor for callers
// that cannot allocate device memory (code under HIP graph capture, serving
// loops, harnesses that forbid hipMalloc).  Its workspace is a file-scope
// device array of fixed size: every device the library runs on holds one copy
// from the first call on that device until the process ends.
//
// The array's name is a host-side stand-in in host code; its device address
// is taken once per device with hipGetSymbolAddress (that device current) and
// only that address is handed to the kernels.
#include <mutex>

#include "../../include/rsvd.h"
#include "internal.hpp"

static __device__ __align__(256) unsigned char scratch[RSVD_NOALLOC_WORKSPACE_BYTES];

namespace {

constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices];   // device address of `scratch` per device (null until the first call there)
std::mutex g_mu;

rsvd_status scratch_on_current_device(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return RSVD_E_HIP;
  if (dev < 0 || dev >= kMaxDevices) return RSVD_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RSVD_E_HIP;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return RSVD_OK;
}

}  // namespace

extern "C" rsvd_status rsvd_factor_noalloc(const rsvd_desc* d, const void* d_A, int64_t lda, const double* d_Omega,
                                           void* d_U, int64_t ldu, double* d_S, void* d_V, int64_t ldv,
                                           void* stream) {
  if (!d || !d_A || !d_U || !d_S) return RSVD_E_ARG;
  if (d->p < 0 || d->q < 0 || d->eps != 0.0 || (d->flags & RSVD_TIMING)) return RSVD_E_ARG;   // fixed rank only
  size_t need = 0;
  rsvd_status s = rsvd_workspace_size(d, &need);
  if (s != RSVD_OK) return s;
  if (need > (size_t)RSVD_NOALLOC_WORKSPACE_BYTES) return RSVD_E_WORKSPACE;
  void* ws = nullptr;
  s = scratch_on_current_device(&ws);
  if (s != RSVD_OK) return s;
  // Nothing in the workspace has to start at zero: the status words the kernels accumulate into are
  // cleared by a fill kernel at the start of every factorisation.
  return (rsvd_status)rsvd::factor_in_workspace(d, ws, (size_t)RSVD_NOALLOC_WORKSPACE_BYTES,
                                                reinterpret_cast<hipStream_t>(stream), d_A, lda, d_Omega, d_U, ldu,
                                                d_S, d_V, ldv);
}
