// FFT-stage kernels instantiated for FP32 (complex64).
#include "k_fft_impl.h"
KFFT_INSTANTIATE(float)
