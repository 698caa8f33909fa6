// Host logic of plan creation that needs no GPU: the neighbour rule's first
// taps (bit-identical to the device's), and the binning of the points into
// tile tasks with their interpolation and spreading orders.  Built into the
// library and, on its own under the address and undefined-behaviour
// sanitizers, into the host test harness.
#include "host_plan.h"

#include <algorithm>
#include <utility>
#include <cmath>
#include <thread>

namespace hostplan {

// ---------------------------------------------------------------------------
// Binning: first tap per axis, bit-identical to the device rule.
#pragma clang fp contract(off)
void host_first_taps(const double* om, int J, int64_t K, double gamma,
                                   int (&first)[3]) {
  for (int d = 0; d < 3; ++d) {
    const double t = om[d] / gamma;
    const double tj = t - 0.5 * (double)J;
    const double k0 = std::floor(tj);
    int64_t f = (int64_t)k0 + 1 + K / 2;
    f %= K;
    if (f < 0) f += K;
    first[d] = (int)f;
  }
}

void point_omega(const BinParams& p, const std::vector<double>& geom, int64_t i,
                 double (&om)[3]) {
  if (p.radial) {
    const int64_t l = i / p.n_r;
    const int64_t c = i - l * p.n_r;
    const double dr = (2.0 * M_PI) / (double)p.n_r;
    const double r = (double)(c - p.n_r / 2) * dr;
    om[0] = r * geom[3 * l + 0];
    om[1] = r * geom[3 * l + 1];
    om[2] = r * geom[3 * l + 2];
  } else {
    om[0] = geom[3 * i + 0];
    om[1] = geom[3 * i + 1];
    om[2] = geom[3 * i + 2];
  }
}
#pragma clang fp contract(on)

// Sort points by the tile of their first tap and cut every bin into tasks of
// at most max_pts points.  Within a task the points are then ordered by the
// LDS bank of their first tap's cell in the staged halo tile, once for each
// of the two kernels that read the order:
//   spreading: points that share their first tap cell are paired (one lane
//     spreads both, summing their contributions to each of the J^3 cells
//     before one LDS atomic); the pairs come first, then the unpaired
//     points (FP32 with Kaiser-Bessel weights; the other kernels spread one
//     point at a time, and their tasks hold no pairs).  Cell
//     c = (l0 S + l1) S + l2 (S = tile + J - 1); pairs, then singles, dealt
//     round-robin over the residues c mod 32, so the lanes of a wave start
//     on distinct banks and a tap offset shared by all lanes keeps them so;
//   interpolation (FP32): rows padded to even pitch S2, cell
//     c = (l0 S + l1) S2 + l2; even cells first, then odd ones (a wave's
//     row reads then share one alignment), each class dealt round-robin over
//     its 16 residues mod 32.  FP64 interpolation uses the spreading order.
// With `twins` (FP32), the two points of a frequency sampled twice (as lines
// in opposite directions sample it: FP64 frequencies that agree to 1e-12,
// relative, and one first tap cell) are linked, kept next to each other in
// the bin and in one task, and paired; their pairs come first in both
// orders: one evaluation of the weights serves both points in spreading, and
// one interpolation both outputs.  Tasks are cut from the bins in point
// order (tasks cut in cell order gathered the coincident omega = 0 samples
// into one task, whose LDS atomics on that one cell serialised: up to 4x
// slower spreading); within each residue the spreading deal takes the points
// in turns over their cells, the interpolation deal in cell order.
void build_bins(const BinParams& p, const std::vector<double>& geom, Binning& B) {
  const int64_t M = p.M;
  const int nb = p.nb, T = p.tile, J = p.J;
  const int S = T + J - 1;
  const bool pairs = p.fp32;
  const bool pair_spread = p.pair_spread;
  const int S2 = pairs ? S + (S & 1) : S;
  const int64_t nbins = (int64_t)nb * nb * nb;
  std::vector<int32_t> key(M);
  std::vector<uint8_t> res_s(M), res_i(M);
  std::vector<uint16_t> lcell(M);  // first tap cell within its tile
  const double gamma = (2.0 * M_PI) / (double)p.K;
  unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (M < 200000) nth = 1;
  auto parallel = [&](int64_t n, auto&& fn) {
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nth; ++t)
      th.emplace_back([&, t]() { fn(n * t / nth, n * (t + 1) / nth); });
    for (auto& t : th) t.join();
  };
  parallel(M, [&](int64_t a, int64_t b) {
    for (int64_t i = a; i < b; ++i) {
      double om[3];
      int first[3];
      point_omega(p, geom, i, om);
      host_first_taps(om, J, p.K, gamma, first);
      key[i] = (int32_t)(((int64_t)(first[0] / T) * nb + first[1] / T) * nb + first[2] / T);
      const int r01 = (first[0] % T) * S + first[1] % T;
      res_s[i] = (uint8_t)((r01 * S + first[2] % T) & 31);
      lcell[i] = (uint16_t)(((first[0] % T) * T + first[1] % T) * T + first[2] % T);
      res_i[i] = (uint8_t)((r01 * S2 + first[2] % T) & 31);
    }
  });
  std::vector<int64_t> off(nbins + 1, 0);
  for (int64_t i = 0; i < M; ++i) off[key[i] + 1]++;
  for (int64_t k = 0; k < nbins; ++k) off[k + 1] += off[k];
  B.perm_s.resize(M);
  {
    std::vector<int64_t> pos(off.begin(), off.end() - 1);
    for (int64_t i = 0; i < M; ++i) B.perm_s[pos[key[i]]++] = (int32_t)i;
  }
  // twins (FP32): within each bin, points put in the order of their first tap
  // cells and frequencies quantised to 2^-30 make the two samples of one
  // frequency neighbours; those whose FP64 frequencies agree to 1e-12
  // (relative) and share the first cell are linked.
  std::vector<int32_t> twin_of(p.twins ? M : 0, -1);
  if (p.twins) {
    struct QKey {
      uint16_t cell;
      int64_t q[3];
      int32_t pt;
    };
    parallel(nbins, [&](int64_t a, int64_t b) {
      std::vector<QKey> qk;
      std::vector<int32_t> order;
      for (int64_t bin = a; bin < b; ++bin) {
        const int64_t s = off[bin], n = off[bin + 1] - s;
        qk.resize(n);
        for (int64_t i = 0; i < n; ++i) {
          double om[3];
          const int32_t pt = B.perm_s[s + i];
          point_omega(p, geom, pt, om);
          qk[i].cell = lcell[pt];
          for (int c = 0; c < 3; ++c) qk[i].q[c] = std::llround(std::ldexp(om[c], 30));
          qk[i].pt = pt;
        }
        std::stable_sort(qk.begin(), qk.end(), [](const QKey& x, const QKey& y) {
          if (x.cell != y.cell) return x.cell < y.cell;
          for (int c = 0; c < 3; ++c)
            if (x.q[c] != y.q[c]) return x.q[c] < y.q[c];
          return false;
        });
        // runs of one cell and quantised frequency (in point order); a run of
        // k points links its first and second halves, point m with point
        // m + k/2: a twin pair for k = 2, and for the frequency every line
        // samples (omega = 0) the samples of opposite lines
        auto same_q = [&](int64_t x, int64_t y) {
          return qk[x].cell == qk[y].cell && qk[x].q[0] == qk[y].q[0] && qk[x].q[1] == qk[y].q[1] &&
                 qk[x].q[2] == qk[y].q[2];
        };
        for (int64_t i = 0; i < n;) {
          int64_t j = i + 1;
          while (j < n && same_q(i, j)) ++j;
          const int64_t h = (j - i) / 2;
          for (int64_t m = 0; m < h; ++m) {
            const int32_t x = qk[i + m].pt, y = qk[i + m + h].pt;
            double oa[3], ob[3];
            point_omega(p, geom, x, oa);
            point_omega(p, geom, y, ob);
            double dmax = 0.0, amax = 1.0;
            for (int c = 0; c < 3; ++c) {
              dmax = std::max(dmax, std::fabs(oa[c] - ob[c]));
              amax = std::max(amax, std::fabs(oa[c]));
            }
            if (dmax <= 1e-12 * amax) {
              twin_of[x] = y;
              twin_of[y] = x;
            }
          }
          i = j;
        }
        // the bin's units (a twin pair, or a point) in the order of their
        // first point: tasks cut from it hold runs of neighbouring lines and
        // of their opposites (whose values share cache lines).  (Coincident
        // samples linked in point order instead of by halves would leave
        // most of the omega = 0 samples of the bin's second half together at
        // its end, in one task whose LDS atomics on that cell serialise.)
        order.clear();
        for (int64_t i = 0; i < n; ++i) {
          const int32_t pt = B.perm_s[s + i], tw = twin_of[pt];
          if (tw < 0 || pt < tw) order.push_back(pt);
        }
        int64_t o = s;
        for (const int32_t pt : order) {
          B.perm_s[o++] = pt;
          if (twin_of[pt] >= 0) B.perm_s[o++] = twin_of[pt];
        }
      }
    });
  }
  B.tasks.clear();
  B.bin_tasks.assign(nbins + 1, 0);
  for (int64_t b = 0; b < nbins; ++b) {
    B.bin_tasks[b] = (int32_t)B.tasks.size();
    const int64_t s = off[b], e = off[b + 1];
    for (int64_t q = s; q < e;) {
      TileTask t;
      t.bin = (int32_t)b;
      t.start = (int32_t)q;
      int64_t n = std::min<int64_t>(p.max_pts, e - q);
      // a task never separates twins
      if (p.twins && n > 1 && q + n < e && twin_of[B.perm_s[q + n - 1]] == B.perm_s[q + n]) --n;
      t.count = (int32_t)n;
      t.npairs = 0;
      t.ntwins = 0;
      B.tasks.push_back(t);
      q += n;
    }
  }
  B.bin_tasks[nbins] = (int32_t)B.tasks.size();
  B.perm = B.perm_s;
  // Reorder pts[0..n) by residue: classes of residues r = cls, cls + step, ...
  // in turn, each dealt round-robin over its residues.
  // With `cell`, each residue's points are first put in the order of their
  // first cells; the spreading (step 1) then takes them in turns over the
  // cells (one point of every cell, then a second of every cell that has
  // one, ...), so that the two points a wave takes from one residue rarely
  // share a cell: lanes adding to the same cell in one LDS atomic are
  // serialised.
  struct Deal {
    std::vector<int32_t> tmp, bucket, cnt = std::vector<int32_t>(33), fill, seg;
    std::vector<std::pair<int, int>> groups;  // (start, size) of each cell's run
    void run(int32_t* pts, int n, const uint8_t* res, int step, const uint16_t* cell = nullptr) {
      std::fill(cnt.begin(), cnt.end(), 0);
      for (int i = 0; i < n; ++i) cnt[res[pts[i]] + 1]++;
      for (int r = 0; r < 32; ++r) cnt[r + 1] += cnt[r];
      tmp.assign(pts, pts + n);
      bucket.resize(n);
      fill.assign(cnt.begin(), cnt.end() - 1);
      for (int i = 0; i < n; ++i) bucket[fill[res[tmp[i]]]++] = tmp[i];
      if (cell)
        for (int r = 0; r < 32; ++r) {
          int32_t* b = bucket.data() + cnt[r];
          const int m = cnt[r + 1] - cnt[r];
          if (m < 2) continue;
          std::stable_sort(b, b + m, [&](int32_t x, int32_t y) { return cell[x] < cell[y]; });
          if (step == 2) continue;  // (interpolation: kept in cell order)
          seg.clear();
          groups.clear();
          for (int i = 0; i < m;) {
            int j = i;
            while (j < m && cell[b[j]] == cell[b[i]]) ++j;
            groups.push_back({i, j - i});
            i = j;
          }
          for (int k = 0; (int)seg.size() < m; ++k)
            for (const auto& g : groups)
              if (k < g.second) seg.push_back(b[g.first + k]);
          std::copy(seg.begin(), seg.end(), b);
        }
      int o = 0;
      for (int cls = 0; cls < step; ++cls) {
        int left = 0;
        for (int r = cls; r < 32; r += step) left += cnt[r + 1] - cnt[r];
        if (step == 2) {
          // groups of 16 points (one LDS pass of 16-byte reads) take one
          // point from each of the 16 fullest residues of the class, so the
          // buckets drain evenly and late groups keep distinct residues
          int rs[16], nr = 0, take[32], rem[32];
          for (int r = cls; r < 32; r += step) {
            rs[nr++] = r;
            take[r] = cnt[r];
            rem[r] = cnt[r + 1] - cnt[r];
          }
          while (left > 0) {
            std::stable_sort(rs, rs + nr, [&](int x, int y) { return rem[x] > rem[y]; });
            int g = 0;
            for (int k = 0; k < nr && g < 16 && rem[rs[k]] > 0; ++k, ++g) {
              pts[o++] = bucket[take[rs[k]]++];
              --rem[rs[k]];
              --left;
            }
            while (g < 16 && left > 0) {  // fewer than 16 residues left
              int best = rs[0];
              for (int k = 1; k < nr; ++k)
                if (rem[rs[k]] > rem[best]) best = rs[k];
              pts[o++] = bucket[take[best]++];
              --rem[best];
              --left;
              ++g;
            }
          }
          continue;
        }
        for (int round = 0; left > 0; ++round)
          for (int r = cls; r < 32; r += step)
            if (cnt[r] + round < cnt[r + 1]) {
              pts[o++] = bucket[cnt[r] + round];
              --left;
            }
      }
    }
  };
  parallel((int64_t)B.tasks.size(), [&](int64_t a, int64_t b) {
    Deal d;
    std::vector<int32_t> sorted, singles, loose, idx, rest;
    std::vector<std::pair<int32_t, int32_t>> twin_pairs, other_pairs;
    std::vector<uint8_t> res_pair;
    std::vector<uint16_t> cell_pair;
    for (int64_t k = a; k < b; ++k) {
      TileTask& t = B.tasks[k];
      int32_t* ps = B.perm_s.data() + t.start;
      if (!pair_spread) {  // no paired spreading: points dealt one by one
        int32_t* pi = B.perm.data() + t.start;  // (still the bin's order)
        if (p.twins) {
          // interpolation order: the task's twin pairs (adjacent in the bin's
          // order), then every other point
          twin_pairs.clear();
          rest.clear();
          for (int i = 0; i < t.count;) {
            if (i + 1 < t.count && twin_of[pi[i]] == pi[i + 1]) {
              twin_pairs.push_back({pi[i], pi[i + 1]});
              i += 2;
            } else {
              rest.push_back(pi[i++]);
            }
          }
          const int nt = (int)twin_pairs.size();
          idx.resize(nt);
          res_pair.resize(nt);
          cell_pair.resize(nt);
          for (int q = 0; q < nt; ++q) {
            idx[q] = q;
            res_pair[q] = res_i[twin_pairs[q].first];
            cell_pair[q] = lcell[twin_pairs[q].first];
          }
          d.run(idx.data(), nt, res_pair.data(), 2, cell_pair.data());
          for (int q = 0; q < nt; ++q) {
            pi[2 * q] = twin_pairs[idx[q]].first;
            pi[2 * q + 1] = twin_pairs[idx[q]].second;
          }
          // spreading order: the twin pairs (one set of weights each), then
          // the rest, each dealt over the residues of their first cells
          for (int q = 0; q < nt; ++q) {
            idx[q] = q;
            res_pair[q] = res_s[twin_pairs[q].first];
          }
          d.run(idx.data(), nt, res_pair.data(), 1, cell_pair.data());
          for (int q = 0; q < nt; ++q) {
            ps[2 * q] = twin_pairs[idx[q]].first;
            ps[2 * q + 1] = twin_pairs[idx[q]].second;
          }
          d.run(rest.data(), (int)rest.size(), res_i.data(), 2, lcell.data());
          std::copy(rest.begin(), rest.end(), pi + 2 * nt);
          d.run(rest.data(), (int)rest.size(), res_s.data(), 1, lcell.data());
          std::copy(rest.begin(), rest.end(), ps + 2 * nt);
          t.ntwins = nt;
          t.npairs = nt;
          continue;
        }
        d.run(pi, t.count, pairs ? res_i.data() : res_s.data(), pairs ? 2 : 1);
        d.run(ps, t.count, res_s.data(), 1, lcell.data());
        t.npairs = 0;
        continue;
      }
      // pair the points of each first tap cell: twins (adjacent in the task's
      // order, so also after the stable sort by cell) with each other, the
      // other points of the cell in their order; the lists then go back to
      // point order, so that points dealt to neighbouring lanes and waves
      // rarely share a cell
      sorted.assign(ps, ps + t.count);
      std::stable_sort(sorted.begin(), sorted.end(),
                       [&](int32_t x, int32_t y) { return lcell[x] < lcell[y]; });
      twin_pairs.clear();
      other_pairs.clear();
      singles.clear();
      for (int i = 0; i < t.count;) {
        int j = i;
        while (j < t.count && lcell[sorted[j]] == lcell[sorted[i]]) ++j;
        loose.clear();
        for (int q = i; q < j;) {
          if (p.twins && q + 1 < j && twin_of[sorted[q]] == sorted[q + 1]) {
            twin_pairs.push_back({sorted[q], sorted[q + 1]});
            q += 2;
          } else {
            loose.push_back(sorted[q++]);
          }
        }
        for (size_t q = 0; q + 1 < loose.size(); q += 2) other_pairs.push_back({loose[q], loose[q + 1]});
        if (loose.size() & 1) singles.push_back(loose.back());
        i = j;
      }
      auto by_first = [](const std::pair<int32_t, int32_t>& x, const std::pair<int32_t, int32_t>& y) {
        return x.first < y.first;
      };
      std::sort(twin_pairs.begin(), twin_pairs.end(), by_first);
      std::sort(other_pairs.begin(), other_pairs.end(), by_first);
      std::sort(singles.begin(), singles.end());
      const int nt = (int)twin_pairs.size(), np = nt + (int)other_pairs.size();
      // spreading order: twin pairs, other pairs, single points, each dealt
      // over the residues of their first cells
      int32_t* o = ps;
      for (const auto* set : {&twin_pairs, &other_pairs}) {
        const int n = (int)set->size();
        idx.resize(n);
        res_pair.resize(n);
        cell_pair.resize(n);
        for (int q = 0; q < n; ++q) {
          idx[q] = q;
          res_pair[q] = res_s[(*set)[q].first];
          cell_pair[q] = lcell[(*set)[q].first];
        }
        d.run(idx.data(), n, res_pair.data(), 1, cell_pair.data());
        for (int q = 0; q < n; ++q) {
          *o++ = (*set)[idx[q]].first;
          *o++ = (*set)[idx[q]].second;
        }
      }
      d.run(singles.data(), (int)singles.size(), res_s.data(), 1, lcell.data());
      std::copy(singles.begin(), singles.end(), o);
      t.npairs = np;
      t.ntwins = nt;
      if (!p.twins) {
        d.run(B.perm.data() + t.start, t.count, pairs ? res_i.data() : res_s.data(), pairs ? 2 : 1);
        continue;
      }
      // interpolation order: the twin pairs (one unit each), then every
      // other point, each dealt over its residues
      int32_t* pi = B.perm.data() + t.start;
      idx.resize(nt);
      res_pair.resize(nt);
      for (int q = 0; q < nt; ++q) {
        idx[q] = q;
        res_pair[q] = res_i[ps[2 * q]];
      }
      cell_pair.resize(nt);
      for (int q = 0; q < nt; ++q) cell_pair[q] = lcell[ps[2 * q]];
      d.run(idx.data(), nt, res_pair.data(), 2, cell_pair.data());
      for (int q = 0; q < nt; ++q) {
        pi[2 * q] = ps[2 * idx[q]];
        pi[2 * q + 1] = ps[2 * idx[q] + 1];
      }
      rest.assign(ps + 2 * nt, ps + t.count);
      d.run(rest.data(), (int)rest.size(), res_i.data(), 2, lcell.data());
      std::copy(rest.begin(), rest.end(), pi + 2 * nt);
    }
  });
}

}  // namespace hostplan
