// Reverse-Grangeat kernels instantiated for FP64 (complex128).
#include "k_grangeat_impl.h"
KGR_INSTANTIATE(double)
