// Staging of global data into LDS tiles with every load of a thread in
// flight at once.
#pragma once

#include "cx.h"

namespace stage {

// Staging of a tile of NE elements by NTH threads: thread t handles elements
// t, t + NTH, ...  Its loads are issued CH at a time before any of them is
// written to LDS, so that they are in flight together (a loop that writes
// each element as it arrives keeps one load per thread in flight and leaves
// the pass bound by memory latency rather than bandwidth); CH bounds the
// registers that hold them.
template <typename T, int NE, int NTH, int CH = (NE + NTH - 1) / NTH, typename Ld, typename St>
__device__ __forceinline__ void tile(int tid, Ld&& ld, St&& st) {
  constexpr int PER = (NE + NTH - 1) / NTH;
#pragma unroll
  for (int k0 = 0; k0 < PER; k0 += CH) {
    cx<T> v[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int idx = tid + (k0 + k) * NTH;
      v[k] = (k0 + k < PER && (NE % NTH == 0 || idx < NE)) ? ld(idx) : cx<T>{0, 0};
    }
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int idx = tid + (k0 + k) * NTH;
      if (k0 + k < PER && (NE % NTH == 0 || idx < NE)) st(idx, v[k]);
    }
  }
}

}  // namespace stage
