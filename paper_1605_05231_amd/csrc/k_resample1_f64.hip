// Method-1 resampling kernels instantiated for FP64 (complex128).
#include "k_resample1_impl.h"
KRS1_INSTANTIATE(double)
