// Plain scan + top-k for callers that cannot allocate device memory (code
// under graph capture, tight serving loops, harnesses that forbid hipMalloc):
// the same count kernel and selection as epi3_scan + epi3_topk with the
// vector-ALU variant, with the workspace taken from a fixed device array of
// this file instead of a caller buffer.
#include <mutex>

#include <hip/hip_runtime.h>

#include "epi3.h"
#include "epi3_internal.h"

namespace {

// The workspace of every call on one GPU.  Each device that loads the library
// holds its own copy until the process ends.  Host code never passes this name
// to a kernel or a copy: it stands for a host-side shadow, and the device
// address comes from hipGetSymbolAddress (static_scratch_ptr below).
static __device__ __align__(256) unsigned char scratch[EPI3_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];  // device address of `scratch`, per device

}  // namespace

namespace epi3 {

// Looks up (once per device) the address of the current device's copy of the
// array.  Called by epi3_init and by the first static call on a device.
int static_scratch_ptr(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return EPI3_E_HIP;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return EPI3_E_HIP;
    g_ptr[dev] = p;
  }
  if (out) *out = g_ptr[dev];
  return EPI3_OK;
}

}  // namespace epi3

extern "C" int epi3_scan_topk_static(const epi3_dataset *d, int32_t k, epi3_hit *hits_host,
                                     int32_t *n_out, void *stream) {
  if (!d || k <= 0 || !hits_host || !n_out) return EPI3_E_INVALID;
  const int64_t need = epi3_workspace_bytes(d, k, EPI3_VARIANT_VALU, 0);
  if (need < 0) return (int)need;
  if (need > (int64_t)EPI3_STATIC_SCRATCH_BYTES) return EPI3_E_WORKSPACE;
  void *ws = nullptr;
  const int rc = epi3::static_scratch_ptr(&ws);
  if (rc != EPI3_OK) return rc;
  // the scan initialises every part of the workspace it reads (selection
  // state, tile queue, key range), so the previous call's contents are harmless
  const int rs = epi3_scan(d, k, EPI3_VARIANT_VALU, 0, ws, EPI3_STATIC_SCRATCH_BYTES, stream);
  if (rs != EPI3_OK) return rs;
  return epi3_topk(d, k, 0, ws, hits_host, n_out, stream);
}
