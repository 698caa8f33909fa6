// FFT-stage kernels instantiated for FP64 (complex128).
#include "k_fft_impl.h"
KFFT_INSTANTIATE(double)
