// static_entry.hip -- fmm_evaluate_static: plan and evaluation in a device
// scratch array the library holds, for callers that cannot allocate device
// memory (code under graph capture, serving loops, harnesses that forbid it).
//
// The array is a file-scope __device__ array of FMM_STATIC_SCRATCH_BYTES; each
// GPU the library runs on holds its own copy until the process ends.  Its
// device address is taken once per device, with that device current, by
// hipGetSymbolAddress on the first call there, and only that address is used
// by host code (the array's name in host code is a host-side stand-in).  The
// host plan object is a per-device static too, so the call allocates nothing.
#include <mutex>

#include "fmm_internal.h"

namespace fmm {
namespace {

constexpr size_t kScratchBytes = FMM_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices];  // device address of scratch, per device
fmm_plan_s g_plan[kMaxDevices];

// Address of this device's scratch array (taken on the first call on it).
hipError_t scratch_of(int dev, char** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return e != hipSuccess ? e : hipErrorInvalidSymbol;
    g_scratch[dev] = p;
  }
  *out = static_cast<char*>(g_scratch[dev]);
  return hipSuccess;
}

}  // namespace
}  // namespace fmm

using namespace fmm;

extern "C" fmm_status fmm_evaluate_static(const fmm_config* cfg, int64_t n, const double* d_pos,
                                          const double* d_q, double* d_phi, double* d_force,
                                          double* d_energy, fmm_stream_t stream,
                                          fmm_plan_t** out_plan) {
  fmm_status st = validate_config_for(cfg);
  if (st != FMM_OK) return st;
  if (!d_pos || !d_q || n < 1 || n > INT32_MAX) return FMM_E_INVALID_ARG;
  Layout lay;
  make_layout(*cfg, n, &lay);
  if (lay.total > kScratchBytes) return FMM_E_WORKSPACE;  // beyond the array's size
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return FMM_E_DEVICE;
  char* ws = nullptr;
  if (scratch_of(dev, &ws) != hipSuccess) return FMM_E_DEVICE;
  fmm_plan_s* P = &g_plan[dev];
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  st = plan_into(P, *cfg, lay, n, d_pos, ws, s, nullptr, false);
  P->is_static = true;
  if (st == FMM_OK) st = evaluate_into(P, d_q, d_phi, d_force, d_energy, s);
  if (out_plan) *out_plan = st == FMM_OK ? P : nullptr;
  return st;
}
