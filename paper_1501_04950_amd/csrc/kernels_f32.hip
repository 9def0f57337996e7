// gfx950 kernels and launchers of libdwa for F32 field storage.
#include "kcommon.h"

namespace dwa {
DWA_INSTANTIATE_PRECISION(F32)
}  // namespace dwa
