// Host construction of the seeded LDGM graph (degree tables, Floyd sampling,
// CSR by coded row, CSC by input).  Pure host code: no HIP call here.
//
// Floating point: the degree weights and thresholds must be reproducible bit
// for bit, so this file is compiled with -ffp-contract=off and uses libm log
// and sqrt only; every sum runs in a fixed order.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>

#include "fs_internal.h"

namespace fs {
namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kTwo53 = 1ull << 53;
constexpr uint64_t kPurposeGraph = 1;

// SplitMix64 output function (Steele, Lea & Flood 2014; Stafford Mix13 constants).
inline uint64_t mix(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

inline uint64_t row_key(uint64_t seed, uint64_t stripe_key, uint64_t row) {
  uint64_t h = mix(seed + kGolden);
  h = mix(h ^ kPurposeGraph);
  h = mix(h ^ stripe_key);
  return mix(h ^ row);
}

inline uint64_t draw(uint64_t key, uint64_t i) { return mix(key + (i + 1) * kGolden); }

// Raptor degree distribution of the paper (§2.2): (degree, Omega_degree).
const std::pair<uint32_t, double> kRaptor[] = {
    {1, 0.007969}, {2, 0.49357},   {3, 0.16622},  {4, 0.072646},  {5, 0.082558},
    {8, 0.056058}, {9, 0.037229},  {19, 0.05559}, {64, 0.025023}, {65, 0.003135},
};

}  // namespace

fs_status degree_weights(const fs_graph_params &p, std::vector<double> &w) {
  const uint32_t k = p.k;
  if (k < 1) return fail(FS_ERR_INVALID, "k must be >= 1");
  w.clear();
  if (p.dist == FS_DIST_RSD) {
    const double c = p.rsd_c, delta = p.rsd_delta;
    if (!(c > 0.0) || !(delta > 0.0 && delta < 1.0))
      return fail(FS_ERR_INVALID, "RSD needs c > 0 and 0 < delta < 1");
    const double R = c * std::log((double)k / delta) * std::sqrt((double)k);
    if (!(R / delta > 1.0)) return fail(FS_ERR_INVALID, "RSD needs R/delta > 1");
    double mf = std::floor((double)k / R);
    uint64_t M = mf < 1.0 ? 1 : (mf > (double)k ? k : (uint64_t)mf);
    w.assign((size_t)k + 1, 0.0);
    // rho(i) + tau(i).  The products i (i - 1) and i k are below 2^41, so
    // forming them in doubles is exact and the branch-free range loops give
    // the same quotients as integer products would (and vectorise).
    const double dk = (double)k;
    auto tau_at = [&](uint64_t i) {
      if (i < M) return R / ((double)i * dk);
      if (i == M) return R * std::log(R / delta) / dk;
      return 0.0;
    };
    w[1] = 1.0 / dk + tau_at(1);
    const uint64_t lo_end = std::min<uint64_t>(M, (uint64_t)k + 1);   // i < M: both terms
    for (uint64_t i = 2; i < lo_end; ++i) {
      const double di = (double)i;
      w[i] = 1.0 / (di * (di - 1.0)) + R / (di * dk);
    }
    if (M >= 2 && M <= k) w[M] = 1.0 / ((double)M * ((double)M - 1.0)) + tau_at(M);
    for (uint64_t i = std::max<uint64_t>(M + 1, 2); i <= k; ++i) {
      const double di = (double)i;
      w[i] = 1.0 / (di * (di - 1.0)) + 0.0;
    }
    return FS_OK;
  }
  std::vector<double> tab;
  if (p.dist == FS_DIST_FINITE) {
    if (p.finite_dmax < 1 || p.finite_w == nullptr)
      return fail(FS_ERR_INVALID, "finite table needs finite_dmax >= 1 and weights");
    tab.assign(p.finite_w, p.finite_w + p.finite_dmax);
  } else if (p.dist == FS_DIST_RAPTOR) {
    tab.assign(65, 0.0);
    for (const auto &e : kRaptor) tab[e.first - 1] = e.second;
  } else {
    return fail(FS_ERR_INVALID, "unknown degree distribution");
  }
  for (double v : tab)
    if (!(v >= 0.0) || std::isinf(v)) return fail(FS_ERR_INVALID, "finite weights must be finite and >= 0");
  const size_t D = std::min<size_t>(tab.size(), k);
  w.assign(D + 1, 0.0);
  double tot = 0.0;
  for (size_t d = 1; d <= D; ++d) {
    w[d] = tab[d - 1];
    tot += w[d];
  }
  if (!(tot > 0.0)) return fail(FS_ERR_INVALID, "finite table has no mass at degrees <= k");
  return FS_OK;
}

fs_status degree_thresholds(const std::vector<double> &w, std::vector<uint64_t> &T) {
  const size_t D = w.size() - 1;
  double W = 0.0;
  for (size_t d = 1; d <= D; ++d) W += w[d];
  T.assign(D, 0);
  // the quotients first (independent, so they vectorise), then the running
  // sum in order; C * 2^53 is never negative, so truncation is the floor
  std::vector<double> q(D + 1);
  for (size_t d = 1; d <= D; ++d) q[d] = w[d] / W;
  double C = 0.0;
  for (size_t d = 1; d < D; ++d) {
    C += q[d];
    const double v = C * (double)kTwo53;
    T[d - 1] = v >= (double)kTwo53 ? kTwo53 : (uint64_t)v;
  }
  if (D) T[D - 1] = kTwo53;
  return FS_OK;
}

fs_status build_host_graph(const fs_graph_params &p, fs_graph &g) {
  if (p.k < 1 || p.n < 1) return fail(FS_ERR_INVALID, "k and n must be >= 1");
  if (p.k > (1u << 20)) return fail(FS_ERR_INVALID, "k above 2^20 is not supported");
  if (p.reserved != 0) return fail(FS_ERR_INVALID, "reserved field must be 0");
  std::vector<double> w;
  fs_status st = degree_weights(p, w);
  if (st != FS_OK) return st;
  std::vector<uint64_t> T;
  degree_thresholds(w, T);

  const uint32_t k = p.k, n = p.n;
  g.k = k;
  g.n = n;
  g.params = p;
  if (p.dist == FS_DIST_FINITE) {
    g.finite_w.assign(p.finite_w, p.finite_w + p.finite_dmax);
    g.params.finite_w = g.finite_w.data();
  } else {
    g.params.finite_w = nullptr;
  }
  // Rows depend only on their own stream, so large graphs are built by
  // several threads over contiguous row ranges, then concatenated in order.
  const uint32_t nthreads = n >= 8192 ? std::min<uint32_t>(8, std::max(1u, std::thread::hardware_concurrency())) : 1;
  std::vector<std::vector<int32_t>> part_col(nthreads);
  std::vector<std::vector<int32_t>> part_deg(nthreads);
  std::vector<uint32_t> part_max(nthreads, 0);
  auto build_rows = [&](uint32_t tid) {
    const uint32_t j0 = (uint32_t)((uint64_t)n * tid / nthreads), j1 = (uint32_t)((uint64_t)n * (tid + 1) / nthreads);
    std::vector<uint32_t> stamp(k, 0xFFFFFFFFu);   // stamp[v] == j: v taken in row j
    std::vector<int32_t> row;
    std::vector<int32_t> &out = part_col[tid];
    std::vector<int32_t> &deg = part_deg[tid];
    deg.reserve(j1 - j0);
    for (uint32_t j = j0; j < j1; ++j) {
      const uint64_t key = row_key(p.seed, p.stripe_key, j);
      const uint64_t v0 = draw(key, 0) >> 11;
      const uint32_t d = (uint32_t)(std::upper_bound(T.begin(), T.end(), v0) - T.begin()) + 1;
      row.clear();
      for (uint32_t s = 0; s < d; ++s) {
        const uint64_t r = (uint64_t)(k - d) + s;
        const uint64_t v = ((draw(key, s + 1) >> 32) * (r + 1)) >> 32;
        const uint32_t pick = (stamp[v] == j) ? (uint32_t)r : (uint32_t)v;
        stamp[pick] = j;
        row.push_back((int32_t)pick);
      }
      std::sort(row.begin(), row.end());
      out.insert(out.end(), row.begin(), row.end());
      deg.push_back((int32_t)d);
      part_max[tid] = std::max(part_max[tid], d);
    }
  };
  if (nthreads == 1) {
    build_rows(0);
  } else {
    std::vector<std::thread> pool;
    for (uint32_t t = 0; t < nthreads; ++t) pool.emplace_back(build_rows, t);
    for (std::thread &th : pool) th.join();
  }
  size_t total = 0;
  for (const auto &pc : part_col) total += pc.size();
  if (total >= (size_t)INT32_MAX) return fail(FS_ERR_INVALID, "graph has 2^31 or more edges");
  g.row_ptr.assign((size_t)n + 1, 0);
  g.col.clear();
  g.col.reserve(total);
  uint32_t max_deg = 0, j = 0;
  for (uint32_t t = 0; t < nthreads; ++t) {
    g.col.insert(g.col.end(), part_col[t].begin(), part_col[t].end());
    for (int32_t d : part_deg[t]) {
      g.row_ptr[j + 1] = g.row_ptr[j] + d;
      ++j;
    }
    max_deg = std::max(max_deg, part_max[t]);
  }
  g.nnz = g.col.size();
  g.max_deg = max_deg;
  auto parallel = [&](auto &&fn) {
    if (nthreads == 1) {
      fn(0u);
      return;
    }
    std::vector<std::thread> pool;
    for (uint32_t t = 0; t < nthreads; ++t) pool.emplace_back(fn, t);
    for (std::thread &th : pool) th.join();
  };
  // transpose by counting sort, rows ascending within a column
  g.col_ptr.assign((size_t)k + 1, 0);
  for (int32_t i : g.col) g.col_ptr[(size_t)i + 1]++;
  uint32_t max_cdeg = 0;
  for (uint32_t i = 0; i < k; ++i) {
    max_cdeg = std::max<uint32_t>(max_cdeg, (uint32_t)g.col_ptr[i + 1]);
    g.col_ptr[i + 1] += g.col_ptr[i];
  }
  g.rowidx.assign(g.nnz, 0);
  g.max_cdeg = max_cdeg;
  // encode segments: rows longer than kSegMax are cut into kSegMax-edge
  // pieces; the pieces are then ordered by length (longest first, ties in
  // row order: a counting sort over lengths 1..kSegMax) and their edges
  // copied into seg_col in that order, so that a tile of consecutive
  // segments holds segments of equal or similar length (the lanes of a wave
  // then finish together) and its edges stay contiguous.
  g.heavy.clear();
  std::vector<uint32_t> by_len(kSegMax + 2, 0);   // segments per length, then start positions
  size_t ns = 0;
  for (uint32_t j = 0; j < n; ++j) {
    const int32_t d = g.row_ptr[j + 1] - g.row_ptr[j];
    if ((uint32_t)d > kSegMax) g.heavy.push_back((int32_t)j);
    const uint32_t full = (uint32_t)d / kSegMax, rest = (uint32_t)d % kSegMax;
    by_len[kSegMax] += full;
    if (rest) by_len[rest]++;
    ns += full + (rest ? 1 : 0);
  }
  // start index of each length, longest first
  std::vector<uint32_t> first(kSegMax + 1, 0);
  uint32_t acc = 0;
  for (uint32_t len = kSegMax; len >= 1; --len) {
    first[len] = acc;
    acc += by_len[len];
  }
  std::vector<int32_t> sbeg(ns);
  g.seg_row.resize(ns);
  g.seg_atomic.resize(ns);
  std::vector<uint32_t> slen(ns);
  for (uint32_t j = 0; j < n; ++j) {
    const int32_t e0 = g.row_ptr[j], e1 = g.row_ptr[j + 1];
    const bool split = (uint32_t)(e1 - e0) > kSegMax;
    for (int32_t e = e0; e < e1; e += (int32_t)kSegMax) {
      const uint32_t len = (uint32_t)(std::min<int32_t>(e1, e + (int32_t)kSegMax) - e);
      const uint32_t at = first[len]++;
      sbeg[at] = e;
      slen[at] = len;
      g.seg_row[at] = (int32_t)j;
      g.seg_atomic[at] = split ? 1 : 0;
    }
  }
  g.nseg = (uint32_t)ns;
  g.seg_ptr.assign(ns + 1, 0);
  for (size_t i = 0; i < ns; ++i) g.seg_ptr[i + 1] = g.seg_ptr[i] + (int32_t)slen[i];
  g.seg_col.resize(g.nnz);
  // thread t fills the CSC columns of its range (scanning every row in
  // order, so rows stay ascending, and writing only its own columns) and
  // copies its share of the segments
  parallel([&](uint32_t t) {
    const uint32_t c0 = (uint32_t)((uint64_t)k * t / nthreads), c1 = (uint32_t)((uint64_t)k * (t + 1) / nthreads);
    std::vector<int32_t> slot(g.col_ptr.begin() + c0, g.col_ptr.begin() + c1);
    for (uint32_t j = 0; j < n; ++j)
      for (int32_t e = g.row_ptr[j]; e < g.row_ptr[j + 1]; ++e) {
        const uint32_t i = (uint32_t)g.col[e];
        if (i >= c0 && i < c1) g.rowidx[slot[i - c0]++] = (int32_t)j;
      }
    const size_t s0 = ns * t / nthreads, s1 = ns * (t + 1) / nthreads;
    for (size_t i = s0; i < s1; ++i)
      std::memcpy(&g.seg_col[g.seg_ptr[i]], &g.col[sbeg[i]], sizeof(int32_t) * slen[i]);
  });
  return FS_OK;
}

}  // namespace fs
