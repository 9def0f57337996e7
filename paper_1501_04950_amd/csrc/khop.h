// The fused hop kernels of one tile size: included only by the per-precision, per-tile
// translation units (kernels_hop_*.hip), which instantiate launch_hop_tile.
#pragma once
#include "kcommon.h"

namespace dwa {

// Ls values with their own compiled kernels; any other Ls <= 32 runs the generic one,
// which is also the only one compiled with the dense fallback (both with 8 sites per
// block, so only the 8-site tile carries them).
template <typename S, int NS, int MODE, int KIND>
int launch_hop_mix_mk(dwa_ctx* ctx, const HopDev& a, dim3 grid, dim3 block, size_t shm) {
#define DWA_HOPMIX(LSV, DV)                                                                        \
  do {                                                                                             \
    if (a.nf > 1)                                                                                  \
      hipLaunchKernelGGL((hop_mix_kernel<S, NS, LSV, MODE, KIND, DV, true>), grid, block, shm, ctx->stream, a); \
    else                                                                                           \
      hipLaunchKernelGGL((hop_mix_kernel<S, NS, LSV, MODE, KIND, DV, false>), grid, block, shm, ctx->stream, a); \
  } while (0)
  const bool dense = use_dense(ctx, S::prec);
  if (hop_specialised(ctx->Ls, dense)) {
    switch (ctx->Ls) {
      case 4: DWA_HOPMIX(4, false); break;
      case 8: DWA_HOPMIX(8, false); break;
      case 12: DWA_HOPMIX(12, false); break;
      default: DWA_HOPMIX(16, false); break;
    }
    return DWA_OK;
  }
  if constexpr (NS == 8) {
    if (dense) DWA_HOPMIX(0, true);
    else DWA_HOPMIX(0, false);
    return DWA_OK;
  }
#undef DWA_HOPMIX
  set_error("fused hop: the generic kernels run 8 sites per block");
  return DWA_EINVAL;
}

template <typename S, int NS>
int launch_hop_tile(dwa_ctx* ctx, const HopDev& a, int mode, int mix, dim3 grid, dim3 block,
                    size_t shm) {
  if (mode == 0 && mix == MIX_N) return launch_hop_mix_mk<S, NS, 0, MIX_N>(ctx, a, grid, block, shm);
  if (mode == 0 && mix == MIX_NT) return launch_hop_mix_mk<S, NS, 0, MIX_NT>(ctx, a, grid, block, shm);
  if (mode == 0 && mix == MIX_GINV_IINV)
    return launch_hop_mix_mk<S, NS, 0, MIX_GINV_IINV>(ctx, a, grid, block, shm);
  if (mode == 0 && mix == MIX_G_BT_G5)
    return launch_hop_mix_mk<S, NS, 0, MIX_G_BT_G5>(ctx, a, grid, block, shm);
  if (mode == 1 && mix == MIX_GINV_IINV)
    return launch_hop_mix_mk<S, NS, 1, MIX_GINV_IINV>(ctx, a, grid, block, shm);
  if (mode == 1 && mix == MIX_G_BT_G5)
    return launch_hop_mix_mk<S, NS, 1, MIX_G_BT_G5>(ctx, a, grid, block, shm);
  if constexpr (S::prec == DWA_F64)
    if (mode == 2 && mix == MIX_GINV_IINV)
      return launch_hop_mix_mk<S, NS, 2, MIX_GINV_IINV>(ctx, a, grid, block, shm);
  set_error("fused hop: unsupported combination of output matrix and epilogue");
  return DWA_EINVAL;
}

}  // namespace dwa

#define DWA_INSTANTIATE_HOP_TILE(S, NS)                                                     \
  namespace dwa {                                                                           \
  template int launch_hop_tile<S, NS>(dwa_ctx*, const HopDev&, int, int, dim3, dim3, size_t); \
  }
