// Evaluation without any device allocation (fmm_evaluate_noalloc): the
// evaluation workspace of one single-vector pass (source records, multipole
// and local expansions, the near field) comes from one file-scope device
// array of kScratchBytes, shared by every plan and call on a device.
#include <mutex>

#include "internal.h"

namespace fmm {
namespace {

constexpr size_t kScratchBytes = (size_t)FMM_NOALLOC_MAX_BYTES;
constexpr int kMaxDevices = 64;

// Each device that runs a kernel of this library holds its own copy until
// the process ends.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {nullptr};

// Device address of the calling thread's current device's scratch array
// (looked up once per device, with that device current).
void* scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) throw Error{FMM_EDEVICE, "device index out of range"};
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw Error{FMM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                   hipGetErrorString(e)};
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}

}  // namespace
}  // namespace fmm

using namespace fmm;

extern "C" fmm_status fmm_evaluate_noalloc(fmm_plan* pl, const void* q, int nrhs, void* pot,
                                           void* field, void* stream) {
  return guard([&] {
    if (!pl) throw Error{FMM_EINVAL, "plan is NULL"};
    if (!q || !pot) throw Error{FMM_EINVAL, "q and pot must not be NULL"};
    if (nrhs < 1 || nrhs > pl->prm.max_rhs) throw Error{FMM_EINVAL, "nrhs out of range"};
    int dev = -1;
    FMM_HIP(hipGetDevice(&dev));
    if (dev != pl->device)
      throw Error{FMM_EDEVICE, "current device differs from the plan's device"};
    const WorkspaceLayout L = workspace_layout(pl->n, pl->nbox, pl->prm, false);
    if (L.forward > kScratchBytes)
      throw Error{FMM_EINVAL, "plan needs " + std::to_string(L.forward) +
                                  " bytes of evaluation workspace; the no-allocation path "
                                  "holds FMM_NOALLOC_MAX_BYTES = " +
                                  std::to_string(kScratchBytes)};
    Workspace ws;
    bind_workspace(ws, (char*)scratch_address(dev), L, 4);
    ws.stages = false;  // stage timing would create events
    evaluate(pl, ws, 0, q, nrhs, pot, field, (hipStream_t)stream);
  });
}
