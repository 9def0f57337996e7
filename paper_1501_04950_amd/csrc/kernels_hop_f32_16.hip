// gfx950 fused hop kernels of libdwa: F32 storage, 16 sites per block.
#include "khop.h"

DWA_INSTANTIATE_HOP_TILE(F32, 16)
