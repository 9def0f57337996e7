// gfx950 fused hop kernels of libdwa: BF16 storage, 16 sites per block.
#include "khop.h"

DWA_INSTANTIATE_HOP_TILE(BF16, 16)
