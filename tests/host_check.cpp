// Test harness for the library's host-side plan logic (no GPU): the neighbour
// rule's first taps, the binning into tile tasks and its two point orders,
// the deapodization, twiddle, Kaiser-Bessel and min-max tables.  Built by
// tests/test_host_plan.py with g++ under the address and undefined-behaviour
// sanitizers, from the library's own host_plan.cpp and tables.cpp.
//
// usage: host_check <in> <out>
//   in : int64 M, K, J, tile, max_pts, n_r, radial, fp32, pair_spread,
//        twins, n_geom, N, n_frac; double beta; double geom[3 n_geom]; double frac[n_frac]
//   out: int32 first[3 M], int32 perm[M], int32 perm_s[M], int64 ntasks,
//        int32 tasks[5 ntasks], int32 bin_tasks[nb^3 + 1], double s[N],
//        double tw[2 K], double psi[J n_frac] (Kaiser-Bessel at the offsets
//        u_j = J/2 - 1 - j + frac), double mm[2 J n_frac] (min-max
//        coefficients, re/im interleaved)
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_1605_05231_amd/csrc/host_plan.h"
#include "../paper_1605_05231_amd/csrc/tables.h"

template <typename V>
static void rd(FILE* f, V* p, size_t n) {
  if (fread(p, sizeof(V), n, f) != n) {
    fprintf(stderr, "short read\n");
    exit(2);
  }
}
template <typename V>
static void wr(FILE* f, const V* p, size_t n) {
  if (n && fwrite(p, sizeof(V), n, f) != n) {
    fprintf(stderr, "short write\n");
    exit(2);
  }
}

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: host_check <in> <out>\n");
    return 2;
  }
  FILE* fi = fopen(argv[1], "rb");
  if (!fi) return 2;
  int64_t h[13];
  rd(fi, h, 13);
  double beta;
  rd(fi, &beta, 1);
  hostplan::BinParams bp;
  bp.M = h[0];
  bp.K = h[1];
  bp.J = (int)h[2];
  bp.tile = (int)h[3];
  bp.max_pts = (int)h[4];
  bp.n_r = h[5];
  bp.radial = h[6] != 0;
  bp.fp32 = h[7] != 0;
  bp.pair_spread = h[8] != 0;
  bp.twins = h[9] != 0;
  bp.nb = (int)(bp.K / bp.tile);
  const int64_t n_geom = h[10], N = h[11], n_frac = h[12];
  std::vector<double> geom(3 * n_geom), frac(n_frac);
  rd(fi, geom.data(), geom.size());
  rd(fi, frac.data(), frac.size());
  fclose(fi);

  std::vector<int32_t> first(3 * bp.M);
  const double gamma = (2.0 * M_PI) / (double)bp.K;
  for (int64_t i = 0; i < bp.M; ++i) {
    double om[3];
    int f[3];
    hostplan::point_omega(bp, geom, i, om);
    hostplan::host_first_taps(om, bp.J, bp.K, gamma, f);
    for (int d = 0; d < 3; ++d) first[3 * i + d] = f[d];
  }
  hostplan::Binning B;
  hostplan::build_bins(bp, geom, B);

  const std::vector<double> s = tables::deapod(N, bp.K, bp.J, beta);
  const std::vector<double> tw = tables::twiddles<double>(bp.K);
  std::vector<double> psi, mm;
  tables::MinMax mmx(N, bp.K, bp.J, s);
  for (double fr : frac) {
    std::vector<std::complex<long double>> c(bp.J);
    mmx.coeffs(fr, c.data());
    for (int j = 0; j < bp.J; ++j) {
      const long double u = 0.5L * bp.J - 1 - j + fr;
      psi.push_back((double)tables::kb_psi(u, bp.J, beta));
      mm.push_back((double)c[j].real());
      mm.push_back((double)c[j].imag());
    }
  }

  FILE* fo = fopen(argv[2], "wb");
  if (!fo) return 2;
  const int64_t ntasks = (int64_t)B.tasks.size();
  wr(fo, first.data(), first.size());
  wr(fo, B.perm.data(), B.perm.size());
  wr(fo, B.perm_s.data(), B.perm_s.size());
  wr(fo, &ntasks, 1);
  wr(fo, reinterpret_cast<const int32_t*>(B.tasks.data()), 5 * B.tasks.size());
  wr(fo, B.bin_tasks.data(), B.bin_tasks.size());
  wr(fo, s.data(), s.size());
  wr(fo, tw.data(), tw.size());
  wr(fo, psi.data(), psi.size());
  wr(fo, mm.data(), mm.size());
  fclose(fo);
  return 0;
}
