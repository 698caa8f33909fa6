// Batched mixed-radix FFTs of length L on tiles held in LDS (gfx950).
//
// A tile holds NL lines of length L.  All NT threads of the workgroup
// cooperate: each Stockham stage reads radix-R butterflies into registers,
// waits, and writes them back in autosorted order, so one LDS buffer serves
// every stage.  Radix plan: as many radix-8 stages as possible, then one
// radix-4 or radix-2, then radix-3 and radix-5 stages (L = 2^a 3^b 5^c).
// Twiddles come from a per-length table tw[i] = exp(-2 pi i i/L) made in FP64
// on the host and rounded once; the inverse transform uses their conjugates.
//
// Layouts:
//   line-major  (LM = true)  element (line, e) at line*pitch + e + e/8; the
//                            1-in-8 pad breaks the stride-R bank conflicts of
//                            the first stage's writes.
//   column-major(LM = false) element (line, e) at e*NL + line; used for strided
//                            axes where NL adjacent columns form one coalesced
//                            row segment of global memory.
#pragma once

#include "cx.h"

namespace fft {

constexpr int count_factor(int n, int f) {
  int c = 0;
  while (n % f == 0) { n /= f; ++c; }
  return c;
}

constexpr bool supported(int L) {
  int n = L;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  while (n % 5 == 0) n /= 5;
  return n == 1 && L % 8 == 0;
}

constexpr int nstages(int L) {
  int e = count_factor(L, 2);
  return e / 3 + (e % 3 ? 1 : 0) + count_factor(L, 3) + count_factor(L, 5);
}

constexpr int radix(int L, int s) {
  int e = count_factor(L, 2);
  int n8 = e / 3, rem = e % 3;
  if (s < n8) return 8;
  s -= n8;
  if (rem) {
    if (s == 0) return rem == 2 ? 4 : 2;
    s -= 1;
  }
  int n3 = count_factor(L, 3);
  if (s < n3) return 3;
  return 5;
}

constexpr int span(int L, int s) {  // product of the radices of stages < s
  int p = 1;
  for (int i = 0; i < s; ++i) p *= radix(L, i);
  return p;
}

template <bool LM, int L, int NL>
__device__ __forceinline__ int addr(int line, int e) {
  if constexpr (LM) {
    return line * (L + L / 8) + e + (e >> 3);
  } else {
    return e * NL + line;
  }
}

template <bool LM, int L, int NL>
constexpr int tile_elems() {
  return LM ? NL * (L + L / 8) : NL * L;
}

// In-register DFT of size R with exponent sign S (-1 forward, +1 inverse).
template <int R, int S, typename T>
__device__ __forceinline__ void dft(cx<T>* a) {
  if constexpr (R == 2) {
    cx<T> t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
  } else if constexpr (R == 4) {
    cx<T> t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
    cx<T> t2 = cadd(a[1], a[3]), t3 = cmul_si<S>(csub(a[1], a[3]));
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, t3);
    a[3] = csub(t1, t3);
  } else if constexpr (R == 8) {
    // even/odd split into two DFT-4 and the W8 twiddles
    cx<T> e[4] = {a[0], a[2], a[4], a[6]};
    cx<T> o[4] = {a[1], a[3], a[5], a[7]};
    dft<4, S>(e);
    dft<4, S>(o);
    const T h = (T)0.70710678118654752440;
    // W8^1 = h (1 + S i), W8^2 = S i, W8^3 = h (-1 + S i)
    cx<T> o1 = {h * (o[1].x - (T)S * o[1].y), h * (o[1].y + (T)S * o[1].x)};
    cx<T> o2 = cmul_si<S>(o[2]);
    cx<T> o3 = {h * (-o[3].x - (T)S * o[3].y), h * (-o[3].y + (T)S * o[3].x)};
    a[0] = cadd(e[0], o[0]);
    a[4] = csub(e[0], o[0]);
    a[1] = cadd(e[1], o1);
    a[5] = csub(e[1], o1);
    a[2] = cadd(e[2], o2);
    a[6] = csub(e[2], o2);
    a[3] = cadd(e[3], o3);
    a[7] = csub(e[3], o3);
  } else if constexpr (R == 3) {
    const T c = (T)0.86602540378443864676;  // sqrt(3)/2
    cx<T> s = cadd(a[1], a[2]);
    cx<T> d = csub(a[1], a[2]);
    cx<T> t = {a[0].x - (T)0.5 * s.x, a[0].y - (T)0.5 * s.y};
    cx<T> r = cmul_si<S>(cscale(d, c));
    a[0] = cadd(a[0], s);
    a[1] = cadd(t, r);
    a[2] = csub(t, r);
  } else if constexpr (R == 5) {
    const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
    const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
    cx<T> a1 = cadd(a[1], a[4]), b1 = csub(a[1], a[4]);
    cx<T> a2 = cadd(a[2], a[3]), b2 = csub(a[2], a[3]);
    cx<T> p1 = {a[0].x + c1 * a1.x + c2 * a2.x, a[0].y + c1 * a1.y + c2 * a2.y};
    cx<T> p2 = {a[0].x + c2 * a1.x + c1 * a2.x, a[0].y + c2 * a1.y + c1 * a2.y};
    cx<T> q1 = cmul_si<S>(cx<T>{s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y});
    cx<T> q2 = cmul_si<S>(cx<T>{s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y});
    a[0] = cadd(a[0], cadd(a1, a2));
    a[1] = cadd(p1, q1);
    a[4] = csub(p1, q1);
    a[2] = cadd(p2, q2);
    a[3] = csub(p2, q2);
  }
}

// One Stockham stage: radix R, span Ns (product of earlier radices).
template <typename T, int L, int NL, int NT, bool LM, int R, int Ns, int S>
__device__ __forceinline__ void stage(cx<T>* buf, const cx<T>* __restrict__ tw, int tid) {
  constexpr int NBL = L / R;
  constexpr int NB = NBL * NL;
  constexpr int PER = (NB + NT - 1) / NT;
  cx<T> v[PER][R];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int b = tid + i * NT;
    if (PER * NT == NB || b < NB) {
      const int line = LM ? b / NBL : b % NL;
      const int j = LM ? b % NBL : b / NL;
#pragma unroll
      for (int q = 0; q < R; ++q) v[i][q] = buf[addr<LM, L, NL>(line, j + q * NBL)];
      if constexpr (Ns > 1) {
        const int k = j % Ns;
#pragma unroll
        for (int q = 1; q < R; ++q) {
          cx<T> w = tw[q * k * (L / (Ns * R))];
          v[i][q] = S < 0 ? cmul(v[i][q], w) : cmulc(v[i][q], w);
        }
      }
      dft<R, S>(v[i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int b = tid + i * NT;
    if (PER * NT == NB || b < NB) {
      const int line = LM ? b / NBL : b % NL;
      const int j = LM ? b % NBL : b / NL;
      const int base = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
      for (int q = 0; q < R; ++q) buf[addr<LM, L, NL>(line, base + q * Ns)] = v[i][q];
    }
  }
  __syncthreads();
}

template <typename T, int L, int NL, int NT, bool LM, int S, int St = 0>
__device__ __forceinline__ void stages(cx<T>* buf, const cx<T>* __restrict__ tw, int tid) {
  if constexpr (St < nstages(L)) {
    stage<T, L, NL, NT, LM, radix(L, St), span(L, St), S>(buf, tw, tid);
    stages<T, L, NL, NT, LM, S, St + 1>(buf, tw, tid);
  }
}

// Transform all NL lines of the tile in place (natural order in and out).
// Callers synchronise before (tile written) — this routine ends synchronised.
template <typename T, int L, int NL, int NT, bool LM, int S>
__device__ __forceinline__ void run(cx<T>* buf, const cx<T>* __restrict__ tw, int tid) {
  stages<T, L, NL, NT, LM, S>(buf, tw, tid);
}

}  // namespace fft
