// Reverse-Grangeat kernels instantiated for FP32 (complex64).
#include "k_grangeat_impl.h"
KGR_INSTANTIATE(float)

bool grangeat_length_supported(int64_t n) {
  switch (n) {
#define CASE(NN) case NN:
    KGR_SIZES(CASE)
#undef CASE
    return true;
    default: return false;
  }
}
