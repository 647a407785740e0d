// nmf_foldin for callers that cannot allocate device memory: the workspace is
// a device array owned by the library (one copy per GPU, held until the
// process ends) instead of a buffer the caller brings.
#include <mutex>

#include "plan_impl.hpp"

using namespace plnmf;

// The array itself.  In host code its name is only a stand-in for the symbol:
// its device address, per GPU, comes from hipGetSymbolAddress below and is
// the only form in which it is handed to kernels or copies.
static __device__ __align__(256) char scratch[NMF_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Device address of `scratch` on device `dev` (the current device), looked up
// once per device.
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(NMF_E_UNSUPPORTED, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(NMF_E_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return NMF_OK;
}

}  // namespace

extern "C" int nmf_foldin_noalloc(nmf_plan p, const nmf_matrix* AnewT, float* Ht_new,
                                  int init_mode, const void* mlp_params, int mlp_hidden,
                                  int max_sweeps, double tol, int* sweeps_done,
                                  double* rel_trace) {
  if (sweeps_done) *sweeps_done = 0;
  if (!p) return fail(NMF_E_ARG, "NULL plan");
  size_t need = 0;
  const int hid = init_mode == NMF_FOLDIN_MLP ? mlp_hidden : 0;
  int rc = nmf_foldin_workspace_bytes(p, AnewT, hid, &need);
  if (rc) return rc;
  if (need > (size_t)NMF_NOALLOC_SCRATCH_BYTES)
    return fail(NMF_E_WORKSPACE,
                "fold-in of %lld documents needs %zu bytes of workspace, more than the "
                "library's %zu-byte device array: split the documents or use nmf_foldin",
                (long long)AnewT->rows, need, (size_t)NMF_NOALLOC_SCRATCH_BYTES);
  int dev = -1;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(NMF_E_HIP, "hipGetDevice failed: %s", hipGetErrorString(e));
  if (dev != p->device)
    return fail(NMF_E_ARG, "current device %d is not the plan's device %d", dev, p->device);
  void* ptr = nullptr;
  rc = scratch_address(dev, &ptr);
  if (rc) return rc;
  return foldin_run(p, AnewT, Ht_new, init_mode, mlp_params, mlp_hidden, max_sweeps, tol,
                    sweeps_done, rel_trace, ptr, (size_t)NMF_NOALLOC_SCRATCH_BYTES);
}
