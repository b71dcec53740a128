// Several independent cells: a cost-model parameter choice per cell
// (fftpim_autotune) and a batch executor that applies many plans together
// (fftpim_batch_*).
//
// Error model (relative L2 error of the potential, rel. to its norm):
//   * near zone (Sec. 3.3): pairs outside the correction ball of radius
//     r_b grid spacings are carried by the order-q grid, whose error falls
//     like r_b^-(q+1) for the 1/r part of G0 and is floored by the
//     interpolation of the oscillation exp(-j k0 r) at (k0 h)^(q+1):
//       e_near = sqrt((A_q r_b^-(q+1))^2 + (B_q (|k0| h)^(q+1))^2);
//   * far zone (Sec. 3.2): G_far is smooth on the scale of the period and of
//     the largest wavenumber kappa = max(|k0|, |k_t|), interpolated at order
//     q_f on spacing D:
//       e_far = max(F_qf (D / L_min)^(qf+1), F'_qf (kappa D)^(qf+1)).
// The constants are fits (with margin) to measured errors of this library
// against exact near-zone sums (uniform cubes, a rod, a closed surface;
// static and k0 h up to 2.5) and of the far zone against exact G_far sums.
//
// Cost model (milliseconds of one apply on one MI355X, fitted to measured
// per-part times): near grid a0 + a1 N (q+1)^3 P + a2 M log2(M) P over the
// padded transform size M; correction c0 + c1 nnz (1 + (P - 1)/4); far zone
// f0 + a1 (2 N + Ngf) (qf+1)^3 P (projection, box moments to nodes,
// interpolation) + the grid sum (Ngf^2 P direct, or the FFT term from 8192
// nodes up).  The parts run concurrently, so the sum ranks
// candidates conservatively.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <exception>
#include <new>
#include <numeric>
#include <random>
#include <vector>

#include "fftpim.h"

namespace {

constexpr double kNearA[9] = {0, 0, 0.10, 0.25, 0.32, 0.55, 1.8, 0, 0};
constexpr double kNearB[9] = {0, 0, 0.048, 0.024, 0.0069, 0.0044, 0.0013, 0, 0};
constexpr double kFarStatic[10] = {0, 0, 0, 0.12, 0, 0.29, 0, 10.0, 0, 0};
constexpr double kFarWave[10] = {0, 0, 0, 0.04, 0, 0.0073, 0, 0.0014, 0, 0};

constexpr double kCostGrid0 = 0.11, kCostGridPt = 1.26e-8, kCostFft = 5.6e-10;
constexpr double kCostCorr0 = 0.06, kCostCorrNnz = 3.6e-9;
constexpr double kCostFar0 = 0.10, kCostFarDirect = 2.0e-9;
constexpr int64_t kFarFftNodes = 8192;
constexpr double kFarMomentBytes = 8.0e9;

int fft_len(int m) {
  int M = 1;
  while (M < m) M *= 2;
  return M;
}

struct Domain {
  int dims;
  double lo[3], hi[3], ext[3];
  double Lmin;
};

struct NearChoice {
  int q = 0, n[3] = {0, 0, 0};
  double rb = 0, err = 0, ms = 1e300;
  int64_t nnz = 0;
};

struct FarChoice {
  int q = 0, n[3] = {0, 0, 0};
  double err = 0, ms = 1e300;
};

// Pairs (observer, source) whose near-grid boxes lie within the ball of
// radius rb spacings (minimum image on periodic axes), estimated from a
// fixed sample of pairs: N^2 times the close fraction.
struct PairSample {
  std::vector<int64_t> obs, src;  // sampled observer and source indices
};

PairSample make_sample(int64_t N, std::mt19937_64& rng) {
  PairSample s;
  const int64_t S1 = std::min<int64_t>(N, 256), S2 = std::min<int64_t>(N, 4096);
  std::uniform_int_distribution<int64_t> pick(0, N - 1);
  s.obs.resize(S1);
  s.src.resize(S2);
  for (int64_t i = 0; i < S1; ++i) s.obs[i] = S1 == N ? i : pick(rng);
  for (int64_t i = 0; i < S2; ++i) s.src[i] = S2 == N ? i : pick(rng);
  return s;
}

int64_t estimate_nnz(const std::vector<double>& xyz, int64_t N, const PairSample& ps, const Domain& d,
                     const int nint[3], const double h[3], double rb) {
  auto boxes = [&](const std::vector<int64_t>& idx) {
    std::vector<int> b(idx.size() * 3);
    for (size_t i = 0; i < idx.size(); ++i)
      for (int c = 0; c < 3; ++c) {
        const int v = static_cast<int>(std::floor((xyz[3 * idx[i] + c] - d.lo[c]) / h[c]));
        b[3 * i + c] = std::min(std::max(v, 0), nint[c] - 1);
      }
    return b;
  };
  const std::vector<int> bo = boxes(ps.obs), bs = boxes(ps.src);
  const double hmax = std::max(h[0], std::max(h[1], h[2]));
  double w[3];
  for (int c = 0; c < 3; ++c) w[c] = h[c] / hmax;
  const double r2 = rb * rb;
  int64_t close = 0;
  for (size_t a = 0; a < ps.obs.size(); ++a)
    for (size_t b = 0; b < ps.src.size(); ++b) {
      double s = 0.0;
      for (int c = 0; c < 3; ++c) {
        int dd = bo[3 * a + c] - bs[3 * b + c];
        if (c < d.dims) {
          const int nc = nint[c];
          if (dd > nc / 2) dd -= nc;
          if (dd < -nc / 2) dd += nc;
        }
        const double x = dd * w[c];
        s += x * x;
      }
      if (s <= r2) ++close;
    }
  const double frac = static_cast<double>(close) / (static_cast<double>(ps.obs.size()) * ps.src.size());
  return static_cast<int64_t>(frac * static_cast<double>(N) * static_cast<double>(N));
}

int tune(const fftpim_problem_t* pr, int64_t N, const double* xyz_dev, double target, int precision, int nrhs,
         fftpim_params_t* out, fftpim_tune_report_t* rep) {
  if (!pr || !xyz_dev || !out || N < 1 || !(target > 0.0) || nrhs < 1) return FFTPIM_ERR_INVALID_ARG;
  if (pr->periodic_dims < 1 || pr->periodic_dims > 3) return FFTPIM_ERR_INVALID_ARG;
  if (precision != FFTPIM_F64 && target < 5e-6) return FFTPIM_ERR_INVALID_ARG;  // FP32 rounding floor
  std::vector<double> xyz(static_cast<size_t>(N) * 3);
  if (hipMemcpy(xyz.data(), xyz_dev, xyz.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return FFTPIM_ERR_DEVICE;
  Domain d{};
  d.dims = pr->periodic_dims;
  d.Lmin = INFINITY;
  for (int c = 0; c < 3; ++c) {
    double mn = INFINITY, mx = -INFINITY;
    for (int64_t i = 0; i < N; ++i) {
      const double v = xyz[3 * i + c];
      if (!std::isfinite(v)) return FFTPIM_ERR_INVALID_ARG;
      mn = std::min(mn, v);
      mx = std::max(mx, v);
    }
    if (c < d.dims) {
      if (!(pr->L[c] > 0.0)) return FFTPIM_ERR_INVALID_ARG;
      if (mn < 0.0 || mx >= pr->L[c]) return FFTPIM_ERR_OUT_OF_CELL;
      d.lo[c] = 0.0;
      d.hi[c] = pr->L[c];
      d.Lmin = std::min(d.Lmin, pr->L[c]);
    } else if (pr->has_box) {
      d.lo[c] = pr->box_lo[c];
      d.hi[c] = pr->box_hi[c];
    } else {
      d.lo[c] = mn;
      d.hi[c] = mx > mn ? mx : mn + 1.0;
    }
    d.ext[c] = d.hi[c] - d.lo[c];
  }
  const double emax = std::max(d.ext[0], std::max(d.ext[1], d.ext[2]));
  const double k0 = std::abs(std::complex<double>(pr->k0, pr->k0_im));
  double kappa = k0;
  for (int c = 0; c < d.dims; ++c) kappa = std::max(kappa, std::abs(std::complex<double>(pr->kt[c], pr->kt_im[c])));
  const bool real_vals = out->value_type == FFTPIM_REAL;
  const int P = real_vals ? (nrhs + 1) / 2 : nrhs;
  std::mt19937_64 rng(12345);
  const PairSample sample = make_sample(N, rng);
  int candidates = 0;

  // the error budget is split between the zones; each side keeps a factor 2
  // against the model
  NearChoice best_near;
  FarChoice best_far;
  double best_ms = 1e300;
  for (double far_share : {0.15, 0.35}) {
    const double e_near = 0.5 * (1.0 - far_share) * target, e_far = 0.5 * far_share * target;
    NearChoice bn;
    for (int q = 2; q <= 6; ++q) {
      for (int m = 6; m <= 512; m = m < 32 ? m + 2 : (m < 128 ? m + 8 : m + 32)) {
        const double hh = emax / m;
        int nint[3], n[3];
        double h[3], hmx = 0;
        bool ok = true;
        for (int c = 0; c < 3; ++c) {
          nint[c] = std::max(1, static_cast<int>(std::ceil(d.ext[c] / hh - 1e-9)));
          h[c] = d.ext[c] / nint[c];
          hmx = std::max(hmx, h[c]);
          n[c] = nint[c] + q + (c < d.dims ? 0 : 1);
          if (n[c] > 2048) ok = false;
        }
        if (!ok) continue;
        const double floor_e = kNearB[q] * std::pow(k0 * hmx, q + 1);
        if (floor_e > 0.7 * e_near) continue;
        const double rest = std::sqrt(e_near * e_near - floor_e * floor_e);
        double rb = std::pow(kNearA[q] / rest, 1.0 / (q + 1));
        rb = std::max(rb, q * std::sqrt(3.0) + 0.01);
        if (rb > 30.0) continue;
        // the ball must stay inside half the cell on periodic axes (one
        // image per side)
        bool fits = true;
        for (int c = 0; c < d.dims; ++c)
          if (rb * hmx > 0.45 * d.ext[c]) fits = false;
        if (!fits) continue;
        double M = 1.0;
        for (int c = 0; c < 3; ++c) M *= fft_len(2 * n[c] - 1);
        const double grid_ms = kCostGrid0 + kCostGridPt * static_cast<double>(N) * std::pow(q + 1, 3) * P +
                               kCostFft * M * std::log2(M) * P + kCostCorr0;
        // the sampled pair count is the costly part of a candidate: skip it
        // when the grid steps alone already cost more than the best so far
        if (grid_ms >= bn.ms) continue;
        ++candidates;
        const int64_t nnz = estimate_nnz(xyz, N, sample, d, nint, h, rb);
        const double ms = grid_ms + kCostCorrNnz * static_cast<double>(nnz) * (1.0 + 0.25 * (P - 1));
        if (ms < bn.ms) {
          bn.q = q;
          for (int c = 0; c < 3; ++c) bn.n[c] = n[c];
          bn.rb = rb;
          bn.err = std::sqrt(std::pow(kNearA[q] * std::pow(rb, -(q + 1)), 2) + floor_e * floor_e);
          bn.ms = ms;
          bn.nnz = nnz;
        }
      }
    }
    FarChoice bf;
    for (int qf : {3, 5, 7}) {
      for (int mf = 2; mf <= 200; ++mf) {
        const double D = emax / mf;
        const double err = std::max(kFarStatic[qf] * std::pow(D / d.Lmin, qf + 1), kFarWave[qf] * std::pow(kappa * D, qf + 1));
        if (err > e_far) continue;
        int nf[3];
        bool ok = true;
        double ngf = 1.0, Mf = 1.0;
        for (int c = 0; c < 3; ++c) {
          const int ni = std::max(1, static_cast<int>(std::ceil(d.ext[c] / D - 1e-9)));
          nf[c] = ni + qf + 1;
          if (nf[c] > 512) ok = false;
          ngf *= nf[c];
          Mf *= fft_len(2 * nf[c] - 1);
        }
        // the far box moments hold (qf+1)^3 values per box and plane
        if (!ok || ngf * std::pow(qf + 1, 3) * P * 16.0 > kFarMomentBytes) break;
        ++candidates;
        const double sum_ms = ngf >= kFarFftNodes ? kCostFft * Mf * std::log2(Mf) * P : kCostFarDirect * ngf * ngf * P;
        const double taps = std::pow(qf + 1, 3);
        const double ms = kCostFar0 + kCostGridPt * (2.0 * static_cast<double>(N) + ngf) * taps * P + sum_ms;
        if (ms < bf.ms) {
          bf.q = qf;
          for (int c = 0; c < 3; ++c) bf.n[c] = nf[c];
          bf.err = err;
          bf.ms = ms;
        }
        break;  // the coarsest grid meeting the budget is the cheapest for this order
      }
    }
    if (bn.q == 0 || bf.q == 0) continue;
    if (bn.ms + bf.ms < best_ms) {
      best_ms = bn.ms + bf.ms;
      best_near = bn;
      best_far = bf;
    }
  }
  if (best_near.q == 0 || best_far.q == 0) return FFTPIM_ERR_UNSUPPORTED;
  for (int c = 0; c < 3; ++c) {
    out->near_n[c] = best_near.n[c];
    out->far_n[c] = best_far.n[c];
  }
  out->near_order = best_near.q;
  out->corr_ball = best_near.rb;
  out->corr_radius = static_cast<int>(std::ceil(best_near.rb));
  out->far_order = best_far.q;
  out->n_images = 1;
  out->precision = precision;
  out->far_sum = FFTPIM_FAR_AUTO;
  if (out->nrhs_max < nrhs) out->nrhs_max = nrhs;
  if (rep) {
    rep->predicted_rel_err = best_near.err + best_far.err;
    rep->predicted_ms = best_ms;
    rep->predicted_corr_nnz = best_near.nnz;
    rep->candidates = candidates;
  }
  return FFTPIM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// batch executor
// ---------------------------------------------------------------------------

struct fftpim_batch_s {
  std::vector<fftpim_plan_t> plans;
  std::vector<double> cost;                 // predicted relative cost per cell
  std::vector<std::vector<int>> lane_cells; // cells of each lane, largest first
  std::vector<hipStream_t> lanes;
  std::vector<hipEvent_t> lane_done;
  hipEvent_t fork = nullptr;
};

namespace {

void batch_free(fftpim_batch_s* b) {
  for (auto s : b->lanes) (void)hipStreamDestroy(s);
  for (auto e : b->lane_done) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  delete b;
}

// Enqueues every cell: fork from the caller's stream to the lanes, each lane
// its cells in turn, join back.
int enqueue(fftpim_batch_s* b, const void* const* in, void* const* out, const int* nrhs, int adjoint,
            hipStream_t st) {
  if (hipEventRecord(b->fork, st) != hipSuccess) return FFTPIM_ERR_DEVICE;
  for (size_t l = 0; l < b->lanes.size(); ++l) {
    if (hipStreamWaitEvent(b->lanes[l], b->fork, 0) != hipSuccess) return FFTPIM_ERR_DEVICE;
    for (int c : b->lane_cells[l]) {
      const int s = adjoint ? fftpim_apply_adjoint(b->plans[c], in[c], out[c], nrhs[c], b->lanes[l])
                            : fftpim_apply(b->plans[c], in[c], out[c], nrhs[c], b->lanes[l]);
      if (s != FFTPIM_OK) return s;
    }
    if (hipEventRecord(b->lane_done[l], b->lanes[l]) != hipSuccess) return FFTPIM_ERR_DEVICE;
  }
  for (size_t l = 0; l < b->lanes.size(); ++l)
    if (hipStreamWaitEvent(st, b->lane_done[l], 0) != hipSuccess) return FFTPIM_ERR_DEVICE;
  return FFTPIM_OK;
}

template <typename F>
int guard(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return FFTPIM_ERR_NO_MEMORY;
  } catch (...) {
    return FFTPIM_ERR_DEVICE;
  }
}

}  // namespace

extern "C" {

int fftpim_autotune(const fftpim_problem_t* problem, int64_t n, const double* xyz_dev, double target_rel_err,
                    int precision, int nrhs, fftpim_params_t* params, fftpim_tune_report_t* report) {
  return guard([&]() { return tune(problem, n, xyz_dev, target_rel_err, precision, nrhs, params, report); });
}

int fftpim_batch_create(fftpim_batch_t* batch, const fftpim_plan_t* plans, int ncells, int nlanes, int use_graph) {
  return guard([&]() -> int {
    if (!batch || !plans || ncells < 1 || nlanes < 1 || nlanes > 16) return FFTPIM_ERR_INVALID_ARG;
    *batch = nullptr;
    // recording the batch as a HIP graph is switched off: its first run
    // ended in a host segmentation fault whose cause is not known
    if (use_graph != 0) return FFTPIM_ERR_UNSUPPORTED;
    fftpim_batch_s* b = new fftpim_batch_s();
    for (int c = 0; c < ncells; ++c) {
      if (!plans[c]) {
        batch_free(b);
        return FFTPIM_ERR_INVALID_ARG;
      }
      fftpim_info_t inf;
      const int s = fftpim_plan_info(plans[c], &inf);
      if (s != FFTPIM_OK) {
        batch_free(b);
        return s;
      }
      // predicted time of one apply (the cost model above, single plane)
      double M = 1.0, ngf = 1.0;
      for (int a = 0; a < 3; ++a) {
        M *= inf.near_fft[a];
        ngf *= inf.far_n[a];
      }
      const double cost = kCostGrid0 + kCostGridPt * inf.n_src * 125.0 + kCostFft * M * std::log2(M) + kCostCorr0 +
                          kCostCorrNnz * static_cast<double>(inf.corr_nnz) + kCostFar0 +
                          (inf.far_fft[0] ? 0.0 : kCostFarDirect * ngf * ngf);
      b->plans.push_back(plans[c]);
      b->cost.push_back(cost);
    }
    // longest processing time first: each cell, largest first, to the lane
    // with the least predicted work so far
    const int L = std::min(nlanes, ncells);
    std::vector<int> order(ncells);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->cost[x] > b->cost[y]; });
    std::vector<double> load(L, 0.0);
    b->lane_cells.assign(L, {});
    for (int c : order) {
      const int l = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
      b->lane_cells[l].push_back(c);
      load[l] += b->cost[c];
    }
    for (int l = 0; l < L; ++l) {
      hipStream_t s;
      hipEvent_t e;
      if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        batch_free(b);
        return FFTPIM_ERR_DEVICE;
      }
      b->lanes.push_back(s);
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        batch_free(b);
        return FFTPIM_ERR_DEVICE;
      }
      b->lane_done.push_back(e);
    }
    if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) {
      batch_free(b);
      return FFTPIM_ERR_DEVICE;
    }
    *batch = b;
    return FFTPIM_OK;
  });
}

int fftpim_batch_apply(fftpim_batch_t b, const void* const* in, void* const* out, const int* nrhs, int adjoint,
                       fftpim_stream_t stream) {
  return guard([&]() -> int {
    if (!b || !in || !out || !nrhs) return FFTPIM_ERR_INVALID_ARG;
    const size_t n = b->plans.size();
    for (size_t c = 0; c < n; ++c)
      if (!in[c] || !out[c] || nrhs[c] < 1) return FFTPIM_ERR_INVALID_ARG;
    return enqueue(b, in, out, nrhs, adjoint != 0, static_cast<hipStream_t>(stream));
  });
}

int fftpim_batch_destroy(fftpim_batch_t b) {
  return guard([&]() -> int {
    if (!b) return FFTPIM_ERR_INVALID_ARG;
    batch_free(b);
    return FFTPIM_OK;
  });
}

}  // extern "C"
