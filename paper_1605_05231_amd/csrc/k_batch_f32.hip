// Batched stage kernels instantiated for FP32 (complex64).
#include "k_batch_impl.h"
KBATCH_INSTANTIATE(float)
