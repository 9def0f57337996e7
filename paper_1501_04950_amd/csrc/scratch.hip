// D_bb (eq.(redblack)) for callers that cannot allocate device memory: the two
// intermediate fields of the operator (the premixed input B G x, black, and the hop
// result N H_rb B G x, red) live in one static device array of the library instead of
// the context's workspace.  Same kernels and launch configuration as dwa_apply_Dbb, so
// the result is bitwise the same.
#include <hip/hip_runtime.h>

#include <mutex>

#include "dwa_internal.h"

namespace dwa {

namespace {

// One array per device, held until the process ends.  In host code `scratch` names a
// host-side stand-in, never the device memory: kernels get the address that
// hipGetSymbolAddress returned for the current device (g_scratch[device]).
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

// Called by dwa_create with the context's device current: look up that device's copy
// of the array once and keep its address.
int scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("device index beyond the static scratch table");
    return DWA_EHIP;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[device]) return DWA_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
  g_scratch[device] = p;
  return DWA_OK;
}

size_t scratch_bytes() { return kScratchBytes; }

}  // namespace dwa

using namespace dwa;

extern "C" int dwa_apply_Dbb_static(dwa_ctx* ctx, int prec, void* out, const void* in) {
  if (!ctx) {
    set_error("null context");
    return DWA_EINVAL;
  }
  if (!ctx->links_set) {
    set_error("links not set (call dwa_set_links first)");
    return DWA_ESTATE;
  }
  if (!out || !in) {
    set_error("null field");
    return DWA_EINVAL;
  }
  if (prec != DWA_F64 && prec != DWA_F32 && prec != DWA_BF16) {
    set_error("bad precision");
    return DWA_EINVAL;
  }
  if (out == in) {
    set_error("out and in must not overlap");
    return DWA_EINVAL;
  }
  const size_t fb = round256(elem_bytes(prec) * field_elems(ctx));
  if (2 * fb > kScratchBytes) {
    set_error("lattice too large for dwa_apply_Dbb_static: two half fields of this precision need " +
              std::to_string(2 * fb) + " bytes, the static scratch holds " + std::to_string(kScratchBytes));
    return DWA_EINVAL;
  }
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (ctx->device >= 0 && ctx->device < kMaxDevices) base = g_scratch[ctx->device];
  }
  if (!base) {
    set_error("static scratch not set up on this device");
    return DWA_EHIP;
  }
  void* tb = base;                                   // B G in (black)
  void* tr = static_cast<unsigned char*>(base) + fb;  // N H_rb B G in (red)
  int rc = launch_smix(ctx, prec, MIX_BG, tb, in, nullptr, 0.0, ctx->Ls, nullptr, nullptr);
  if (rc != DWA_OK) return rc;
  const HopOp a{tb, tr, nullptr, nullptr, 1.0, 0.0, 0.0, MIX_N, 1, ctx->Ls, nullptr, 1};
  if ((rc = launch_hop(ctx, prec, a, nullptr)) != DWA_OK) return rc;
  const HopOp b{tr, out, nullptr, in, -0.25, 0.0, 1.0, MIX_GINV_IINV, 0, ctx->Ls, nullptr, 1};
  return launch_hop(ctx, prec, b, nullptr);
}
