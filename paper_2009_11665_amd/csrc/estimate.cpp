// (eps, delta) driver of the colour-coding estimator (Alg. 1; Sec. 2.2.2).
//
// Alg. 1 runs N = O(e^k log(1/delta) / eps^2) random colourings and outputs
// the average of the per-colouring estimates colourful / (P alpha); the
// constant of the O(.) is not given.  Here it is fixed by the standard
// median-of-means argument: every per-colouring estimate X lies in
// [0, emb / P] and has mean emb, so Var X <= emb^2 (1/P - 1); the mean of
// m = ceil(4 (1/P - 1) / eps^2) colourings is off by more than eps * emb with
// probability at most 1/4 (Chebyshev), and the median of r = ceil(8 ln(1/delta))
// such group means is off with probability at most delta (Hoeffding on the
// number of bad groups).  N = r m <= 32 e^k ln(1/delta) / eps^2 since
// 1/P <= e^k for k = t.  Host-only: every colouring is counted by sg2v_count.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "internal.h"

using namespace sg2v;

namespace {

// z with P(|Z| > z) = a for a standard normal Z, by bisection on erfc.
double normal_two_sided(double a) {
  double lo = 0.0, hi = 40.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (std::erfc(mid / std::sqrt(2.0)) > a) lo = mid;
    else hi = mid;
  }
  return 0.5 * (lo + hi);
}

}  // namespace

extern "C" sg2v_status sg2v_estimate(const sg2v_plan *plan, const sg2v_graph *g, uint64_t seed,
                                     double eps, double delta, sg2v_mode mode,
                                     int64_t max_colorings, uint32_t flags, void *stream,
                                     sg2v_estimate_t *out, double *trace) {
  if (!plan || !g || !out || !(eps > 0.0) || !(delta > 0.0 && delta < 1.0) ||
      (flags & ~SG2V_ESTIMATE_ADAPTIVE)) {
    set_error("sg2v_estimate: null handle, eps <= 0, delta outside (0, 1) or unknown flag");
    return SG2V_EINVAL;
  }
  const Plan &P = plan->p;
  const double inv_p = 1.0 / P.P;
  const double m_real = std::ceil(4.0 * std::max(inv_p - 1.0, 0.0) / (eps * eps));
  const double r_real = std::ceil(8.0 * std::log(1.0 / delta));
  const int64_t m = std::max<int64_t>(1, (int64_t)std::min(m_real, 1e15));
  const int64_t r = std::max<int64_t>(1, (int64_t)r_real);
  const double n_bound = (double)m * (double)r;
  const int64_t limit = max_colorings > 0 ? max_colorings : ((int64_t)1 << 24) - 1;
  if (limit >= ((int64_t)1 << 24)) {
    set_error("sg2v_estimate: at most 2^24 - 1 colourings per seed");
    return SG2V_ERANGE;
  }
  // a cap below the bound keeps the r groups and shrinks each
  const int64_t total = (int64_t)std::min<double>(n_bound, (double)limit);
  const int64_t groups = std::min<int64_t>(r, total);
  const int64_t per_group = std::max<int64_t>(1, total / groups);
  const double z = normal_two_sided(delta);

  std::vector<double> est;
  est.reserve((size_t)std::min<int64_t>(total, 1 << 22));
  std::vector<double> group_mean;
  double sum = 0.0, sumsq = 0.0;
  int stopped = 0;
  // colourings per sg2v_count call: at most 4096 and 256 MB of colours
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(4096, ((int64_t)1 << 28) / std::max<int64_t>(1, graph_vertices(g))));
  int64_t done = 0;
  for (int64_t q = 0; q < groups; ++q) {
    double gs = 0.0;
    for (int64_t j = 0; j < per_group; j += chunk) {
      const int32_t cnt = (int32_t)std::min<int64_t>(chunk, per_group - j);
      sg2v_colorings *c = nullptr;
      sg2v_status st = sg2v_color(g, P.k, seed, (int32_t)done, cnt, stream, &c);
      if (st != SG2V_OK) return st;
      std::vector<double> e(cnt);
      st = sg2v_count(plan, g, c, mode, stream, nullptr, nullptr, e.data(), nullptr, nullptr);
      sg2v_colorings_destroy(c);
      if (st != SG2V_OK) return st;
      for (double v : e) {
        gs += v;
        sum += v;
        sumsq += v * v;
        est.push_back(v);
      }
      done += cnt;
    }
    group_mean.push_back(gs / (double)per_group);
    if (trace) trace[q] = sum / (double)done;
    if ((flags & SG2V_ESTIMATE_ADAPTIVE) && q >= 1) {
      const double mean = sum / (double)done;
      const double var = std::max(0.0, (sumsq - sum * mean) / (double)(done - 1));
      if (mean > 0.0 && z * std::sqrt(var / (double)done) <= eps * mean) {
        stopped = 1;
        break;
      }
    }
  }
  const double N = (double)done;
  const double mean = sum / N;
  // sample variance by a second pass (the one-pass form only steers the stop)
  double ss = 0.0;
  for (double v : est) ss += (v - mean) * (v - mean);
  const double var = done > 1 ? ss / (N - 1.0) : 0.0;
  std::vector<double> gm = group_mean;
  std::sort(gm.begin(), gm.end());
  const size_t h = gm.size();
  const double median = h % 2 ? gm[h / 2] : 0.5 * (gm[h / 2 - 1] + gm[h / 2]);
  out->n_colorings = done;
  out->n_bound = (int64_t)std::min(n_bound, 9.0e18);
  out->group_size = per_group;
  out->groups = (int32_t)group_mean.size();
  out->mean = mean;
  out->median_of_means = median;
  out->variance = var;
  out->std_error = std::sqrt(var / N);
  out->ci_low = mean - z * out->std_error;
  out->ci_high = mean + z * out->std_error;
  out->rel_half_width = mean != 0.0 ? z * out->std_error / std::fabs(mean) : INFINITY;
  out->stopped_early = stopped;
  out->capped = (double)done < n_bound && !stopped ? 1 : 0;
  return SG2V_OK;
}
