// Batched stage kernels instantiated for FP64 (complex128).
#include "k_batch_impl.h"
KBATCH_INSTANTIATE(double)
