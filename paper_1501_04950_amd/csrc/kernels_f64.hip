// gfx950 kernels and launchers of libdwa for F64 field storage.
#include "kcommon.h"

namespace dwa {
DWA_INSTANTIATE_PRECISION(F64)
}  // namespace dwa
