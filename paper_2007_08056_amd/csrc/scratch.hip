// The library's own device workspace for symtensor_contract_static: one
// file-scope device array per device the library runs on, set up once per
// device by symtensor_create and held until the process ends.
//
// In host code `scratch` names a host-side stand-in, not device memory; its
// device address on each device comes from hipGetSymbolAddress (called with
// that device current) and is the only form of it ever handed to a kernel or
// a copy.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "symtensor.h"

namespace symt {

namespace {

static __device__ __align__(256) unsigned char scratch[SYMT_STATIC_WORKSPACE_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

// Resolves the array's address on `device` (which must be current) once;
// returns a SYMT_* status.
int scratch_setup(int device, std::string* err) {
  if (device < 0 || device >= kMaxDevices) {
    if (err) *err = "device index above the library's limit of 64";
    return SYMT_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_ptr[device]) return SYMT_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    if (err) *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    return SYMT_EHIP;
  }
  g_ptr[device] = p;
  return SYMT_OK;
}

// Device address of the array on `device`, or nullptr before scratch_setup.
void* scratch_device_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  return g_ptr[device];
}

}  // namespace symt
