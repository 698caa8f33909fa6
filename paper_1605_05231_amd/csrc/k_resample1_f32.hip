// Method-1 resampling kernels instantiated for FP32 (complex64).
#include "k_resample1_impl.h"
KRS1_INSTANTIATE(float)

bool resample1_length_supported(int64_t n) {
  switch (n) {
#define CASE(NN) case NN:
    KRS1_SIZES(CASE)
#undef CASE
    return true;
    default: return false;
  }
}
