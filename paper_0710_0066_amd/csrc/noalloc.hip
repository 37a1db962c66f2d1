// Allocation-free entry point: the x0 force profile with its chunk partials in one fixed
// file-scope device array per GPU instead of the context's workspace, and its result left
// in device memory, so that a caller under HIP graph capture or in a loop that must not
// allocate can use it. The kernels are those of sap_force_profile.
#include <mutex>
#include "force.h"

using namespace sap;

namespace {

// Partial sums of the profile kernel: 2 * L0 * ceil(V3 / 256) doubles (two per slice and
// chunk of 128 sites of one parity). 2 MiB holds e.g. a 64^3 x 128 lattice.
constexpr size_t kScratchDoubles = (size_t)1 << 18;
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices];   // device address of `scratch` on each GPU, or null

}  // namespace

// Resolve the device address of `scratch` on `device`, which must be current; once per
// device (later calls return at once). Called by sap_create.
int sap_noalloc_setup(sap_ctx* c) {
  if (c->device < 0 || c->device >= kMaxDevices)
    return sap_fail(c, SAP_E_HIP, "device index beyond the allocation-free entry's table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[c->device]) return SAP_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return sap_fail(c, SAP_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[c->device] = (double*)p;
  return SAP_OK;
}

extern "C" {

size_t sap_force_profile_noalloc_max(void) { return kScratchDoubles; }

int sap_force_profile_noalloc(sap_ctx* c, const double* F, double* prof, void* stream) {
  if (!c) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (!F || !prof) return sap_fail(c, SAP_E_ARG, "F or prof is NULL");
  const size_t need = (size_t)2 * c->geom.L[0] * (size_t)force_profile_nck(c->g);
  if (need > kScratchDoubles)
    return sap_fail(c, SAP_E_ARG, "lattice too large for the allocation-free force profile: needs " +
                                      std::to_string(need) + " partial sums, the fixed array holds " +
                                      std::to_string(kScratchDoubles));
  double* part;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    part = (c->device >= 0 && c->device < kMaxDevices) ? g_scratch_ptr[c->device] : nullptr;
  }
  if (!part) return sap_fail(c, SAP_E_STATE, "scratch address not resolved for this device");
  launch_force_profile(c->g, F, part, prof, (hipStream_t)stream);
  SAP_HIP_CHECK(c, hipGetLastError());
  return SAP_OK;
}

}  // extern "C"
