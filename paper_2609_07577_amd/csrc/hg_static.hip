// Connectivity (Section 3, Eq. 1) with no allocation: the scratch of the
// connectivity kernels lives in a fixed device array of the library instead
// of the context's arena, for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops).
//
// The array is a file-scope __device__ variable; host code never passes its
// name to a kernel (on the host that name is a stand-in, not a device
// address).  hg_create looks its address up once per device, with that
// device current, and every later use goes through the looked-up address.
// Each GPU the library runs on holds one array of kStaticScratchBytes until
// the process ends; every call on that GPU shares it, so calls that overlap
// on one GPU (two streams, two host threads) race and must be serialised by
// the caller.  The kernels clear what must start at zero (counters, bitmap
// words) themselves on every call.
#include <mutex>

#include "hg_host.h"

namespace hg {
namespace {

constexpr size_t kStaticScratchBytes = 64ull << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kStaticScratchBytes];

std::mutex g_mu;
char* g_ptr[kMaxDevices] = {};
hipError_t g_state[kMaxDevices] = {};  // result of the lookup on each device
bool g_done[kMaxDevices] = {};

}  // namespace

int static_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return HG_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_done[device]) return g_state[device] == hipSuccess ? HG_OK : HG_ERR_HIP;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) (void)hipGetLastError();
  g_state[device] = e;
  g_ptr[device] = e == hipSuccess ? static_cast<char*>(p) : nullptr;
  g_done[device] = true;
  return e == hipSuccess ? HG_OK : HG_ERR_HIP;
}

}  // namespace hg

using namespace hg;

extern "C" {

int hg_connectivity_static(hg_ctx* c, const hg_level* lvl, const int32_t* part, int64_t* conn) {
  if (!c) return HG_ERR_INVALID_ARG;
  int rc = check_level(c, lvl, false);
  if (rc) return rc;
  if ((lvl->n_vertices > 0 && !part) || !conn) return fail(c, HG_ERR_INVALID_ARG, "null argument");
  const size_t need = connectivity_scratch_bytes(lvl->n_vertices, lvl->n_edges);
  if (need > kStaticScratchBytes)
    return fail(c, HG_ERR_CAPACITY,
                "hg_connectivity_static: the level needs %zu bytes of scratch, above the fixed "
                "maximum of %zu (12 bytes per vertex and 16 per hyperedge); use hg_connectivity",
                need, kStaticScratchBytes);
  char* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (c->device >= 0 && c->device < kMaxDevices && g_done[c->device])
      base = g_ptr[c->device];
  }
  if (!base)
    return fail(c, HG_ERR_HIP, "hg_connectivity_static: no fixed scratch on device %d",
                c->device);
  if (c->validate && (rc = validate_with(c, lvl, base)) != HG_OK) return rc;
  return run_connectivity(c, lvl, part, conn, base);
}

}  // extern "C"
