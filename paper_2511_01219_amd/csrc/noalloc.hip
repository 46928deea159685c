// reloc_relocalize without any allocation: for callers that cannot
// allocate device memory (code under stream capture, tight serving loops,
// hosts that forbid allocation after start-up).
//
// Every device buffer of the request (its tables, the per-hypothesis work
// buffers, the sort scratch, the result rows) is carved out of one
// file-scope device array of kScratchBytes. Each GPU the library runs on
// holds its own copy of the array until the process ends; its address on a
// device is looked up once, when a context is created on that device, and
// kept per device. The host name of the array is only a stand-in for the
// symbol: host code never passes it to a kernel or a copy, only the looked-up
// address. Every call on one GPU shares that GPU's copy, so calls that
// overlap on one GPU (from different contexts) race; the kernels clear every
// word they later read (the per-rank best words in the coarse kernel, the
// refinement words in the selection kernel), so nothing depends on what an
// earlier call left there.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "reloc.h"
#include "runtime_internal.h"

namespace {
constexpr size_t kScratchBytes = (size_t)64 << 20;
}  // namespace

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace reloc {

namespace {
std::mutex g_mu;
constexpr int kMaxDevices = 64;
uint8_t* g_ptr[kMaxDevices] = {};
}  // namespace

int32_t noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices)
    return fail(RELOC_E_DEVICE, "device %d beyond the %d the library tracks", device,
                kMaxDevices);
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return RELOC_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(RELOC_E_DEVICE, "no-allocation scratch address on device %d: %s", device,
                hipGetErrorString(e));
  g_ptr[device] = (uint8_t*)p;
  return RELOC_OK;
}

}  // namespace reloc

using namespace reloc;

extern "C" int32_t reloc_relocalize_noalloc(reloc_ctx* c, int32_t map_id, int32_t set_id,
                                            const reloc_scan* scan,
                                            const reloc_search_params* params, reloc_pose* out,
                                            int32_t cap, int32_t* n_out, reloc_stats* st) {
  if (n_out) *n_out = 0;
  if (!c || !n_out || (!out && cap > 0)) return fail(RELOC_E_INVALID, "null argument");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  uint8_t* base = nullptr;
  {
    std::lock_guard<std::mutex> g(g_mu);
    if (c->device >= 0 && c->device < kMaxDevices) base = g_ptr[c->device];
  }
  if (!base) return fail(RELOC_E_DEVICE, "no-allocation scratch not set up on this device");
  RELOC_GUARD_BEGIN
  Request R;
  if (int32_t e = init_request(c, map_id, set_id, scan, params, &R)) return e;
  if (int32_t e = set_device(c)) return e;
  R.carve_base = base;
  R.carve_cap = kScratchBytes;
  if (int32_t e = build_request(c, R)) return e;   // carves; nothing to release
  PoseRow* rows = req_alloc<PoseRow>(c, R, (size_t)R.rows_cap);
  if (!rows) return RELOC_E_NOMEM;
  return run_request(c, R, out, cap, n_out, st, rows);
  RELOC_GUARD_END
}
