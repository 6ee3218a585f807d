// pr_render_views_static: pr_render_views with its frame work area (frame
// header, runs, per-(batch, view) render records) in a device array of fixed
// size that the library holds, instead of a caller-owned work buffer.  For
// callers that cannot allocate device memory on the frame path.
//
// The array is a file-scope __device__ variable: every GPU the library runs on
// holds its own copy, at its own address, from the library's first use on that
// device until the process ends.  Host code never passes the variable's name
// to a kernel (in host code it is only a stand-in, not a device address): at
// pr_create, with the context's device current, hipGetSymbolAddress gives the
// device address, which is kept per device and used from then on.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/ptraster.h"
#include "internal.h"

namespace {

static __device__ __align__(256) uint8_t scratch[PR_STATIC_WORK_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices];  // device address of scratch per device ordinal (null: not looked up yet)

}  // namespace

namespace ptr {

// Looks up this device's copy of the array (once per device).  The caller has
// made `device` current.
hipError_t static_work_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_addr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_addr[device] = p;
  return hipSuccess;
}

void* static_work_addr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  return g_addr[device];
}

}  // namespace ptr
