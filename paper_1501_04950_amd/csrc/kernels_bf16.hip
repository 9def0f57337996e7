// gfx950 kernels and launchers of libdwa for BF16 field storage.
#include "kcommon.h"

namespace dwa {
DWA_INSTANTIATE_PRECISION(BF16)
}  // namespace dwa
