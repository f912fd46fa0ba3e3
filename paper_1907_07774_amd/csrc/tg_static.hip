// tg_forward_static: the forward solve with the plan's workspace in a
// static device array of the library, for callers that cannot allocate
// device memory (graph capture, serving loops, harnesses without hipMalloc).
//
// The array `scratch` lives in this file's code object.  In host code its
// name is only a host-side stand-in: its device address differs per device
// and is looked up once per device with hipGetSymbolAddress, then only that
// address is handed to the plan (and so to every kernel).
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/tumorgrad.h"
#include "tg_internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[TG_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

struct Slot {
  void* ptr = nullptr;       // device address of `scratch` on this device
  tg_plan* owner = nullptr;  // plan currently bound to it
};

std::mutex g_mu;
Slot g_slot[kMaxDevices];

// Forget `plan` as owner on every device (caller holds g_mu).
void release_locked(tg_plan* plan) {
  for (Slot& s : g_slot)
    if (s.owner == plan) s.owner = nullptr;
}

}  // namespace

namespace tg {
void static_scratch_release(tg_plan* plan) {
  std::lock_guard<std::mutex> lk(g_mu);
  release_locked(plan);
}
}  // namespace tg

extern "C" tg_status tg_forward_static(tg_plan* plan, const double* d_p, const double* d_rho_f,
                                       const double* d_k_f, const void* d_m, void* d_cT,
                                       void* stream) {
  if (plan == nullptr || d_p == nullptr || d_rho_f == nullptr || d_k_f == nullptr ||
      d_m == nullptr || d_cT == nullptr)
    return TG_ERR_ARG;
  size_t need = 0;
  if (tg_plan_workspace_bytes(plan, &need) != TG_OK) return TG_ERR_ARG;
  if (need > TG_STATIC_SCRATCH_BYTES) return TG_ERR_SCRATCH_LIMIT;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return TG_ERR_HIP;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    Slot& s = g_slot[dev];
    if (s.ptr == nullptr) {
      // once per device, with that device current
      void* p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
        return TG_ERR_HIP;
      s.ptr = p;
    }
    if (s.owner != plan || tg::plan_workspace(plan) != s.ptr) {
      if (s.owner != nullptr && s.owner != plan) tg::plan_unbind(s.owner);
      release_locked(plan);
      s.owner = nullptr;
      const tg_status st = tg::plan_bind_ws(plan, s.ptr, TG_STATIC_SCRATCH_BYTES);
      if (st != TG_OK) return st;
      s.owner = plan;
    }
  }
  return tg_forward(plan, d_p, d_rho_f, d_k_f, d_m, d_cT, stream);
}
