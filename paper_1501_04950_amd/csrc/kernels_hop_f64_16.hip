// gfx950 fused hop kernels of libdwa: F64 storage, 16 sites per block.
#include "khop.h"

DWA_INSTANTIATE_HOP_TILE(F64, 16)
