// Interpolation / spreading kernels instantiated for FP64 (complex128).
#include "k_grid_impl.h"
KGRID_INSTANTIATE(double)
