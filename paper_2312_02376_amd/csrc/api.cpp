// C ABI of the FFT-PIM apply: plan construction (Sec. 3.2-3.3 preprocessing)
// and the apply / conjugate-transpose orchestration.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <stdexcept>
#include <system_error>
#include <thread>
#include <vector>

#include "kernels.h"

using namespace fftpim;

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxNearOrder = 8;
constexpr int kMaxFarOrder = 9;
constexpr int kMaxCorrRadius = 40;
constexpr size_t kLdsBudget = 64 * 1024;
// planes up to which the near projection runs through the node-major weight CSR
constexpr int kSpreadCsrPlanes = 4;

#define HIPCHK(expr)                                  \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) {                           \
      if (e_ == hipErrorOutOfMemory) return FFTPIM_ERR_NO_MEMORY; \
      return FFTPIM_ERR_DEVICE;                       \
    }                                                 \
  } while (0)

#define CHK(expr)               \
  do {                          \
    int s_ = (expr);            \
    if (s_ != FFTPIM_OK) return s_; \
  } while (0)

// AUTO far sum: the FFT convolution from this many far grid nodes up
constexpr int64_t kFarFftMinNodes = 8192;
// smallest transform length (a power of two) holding m points
int fft_length(int m) {
  int M = 1;
  while (M < m) M *= 2;
  return M;
}
int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Device allocation owned by the plan; refused (NO_MEMORY) when it would take
// the plan's device memory beyond params.max_bytes (0 = no limit).
template <typename T>
int dalloc(fftpim_plan_s* p, T** out, size_t count) {
  void* ptr = nullptr;
  size_t bytes = std::max<size_t>(count * sizeof(T), 16);
  if (p->prm.max_bytes != 0 && static_cast<uint64_t>(p->device_bytes) + bytes > p->prm.max_bytes)
    return FFTPIM_ERR_NO_MEMORY;
  if (hipMalloc(&ptr, bytes) != hipSuccess) return FFTPIM_ERR_NO_MEMORY;
  p->allocations.push_back(DevBuf{ptr, bytes});
  p->device_bytes += static_cast<int64_t>(bytes);
  *out = static_cast<T*>(ptr);
  return FFTPIM_OK;
}

void dfree(fftpim_plan_s* p, void* ptr) {
  if (!ptr) return;
  auto it = std::find_if(p->allocations.begin(), p->allocations.end(), [&](const DevBuf& b) { return b.p == ptr; });
  if (it != p->allocations.end()) {
    p->device_bytes -= static_cast<int64_t>(it->bytes);
    p->allocations.erase(it);
    (void)hipFree(ptr);
  }
}

template <typename T>
int upload(fftpim_plan_s* p, T** out, const std::vector<T>& host) {
  CHK(dalloc(p, out, host.size()));
  if (!host.empty()) HIPCHK(hipMemcpy(*out, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice));
  return FFTPIM_OK;
}

size_t cbytes(const fftpim_plan_s* p) { return p->prm.precision != FFTPIM_F64 ? 8 : 16; }

// The correction region of Eq. (er) over box offsets: its per-axis reach (in
// boxes) and, for the ball, the weights h_c / h_max and the squared radius
// (with a relative slack of 1e-9 that settles offsets on the sphere).
struct CorrRegion {
  int reach[3];
  int ball;
  double bw[3], br2;
};

CorrRegion corr_region(const fftpim_plan_s* p) {
  CorrRegion r{};
  const double rb = p->prm.corr_ball;
  r.ball = rb > 0.0 ? 1 : 0;
  const double hmax = std::max(p->ng.h[0], std::max(p->ng.h[1], p->ng.h[2]));
  for (int c = 0; c < 3; ++c) {
    r.bw[c] = p->ng.h[c] / hmax;
    r.reach[c] = r.ball ? static_cast<int>(std::floor(rb / r.bw[c] * (1.0 + 1e-9))) : p->prm.corr_radius;
  }
  r.br2 = rb * rb * (1.0 + 1e-9);
  return r;
}

// Stencil start and offset for one coordinate on a grid (Sec. 3.2, Eq. (grid),
// with the halo reading): t = (x - origin)/h, s = floor(t - (q-1)/2) clamped
// to [0, n-1-q], u = t - s.
void stencil(double x, double origin, double h, int q, int n, int32_t& s, double& u) {
  double t = (x - origin) / h;
  double sf = std::floor(t - 0.5 * (q - 1));
  int si = static_cast<int>(sf);
  si = std::max(0, std::min(n - 1 - q, si));
  s = si;
  u = t - si;
}

// 1D Lagrange weights of the q+1 stencil nodes at offset u (Sec. 3.2, the
// q-th order interpolation of Eq. (PGF_interp)), as a [3][q+1][N] array.
std::vector<double> weights_soa(const std::vector<double>& u_soa, int64_t N, int q) {
  std::vector<double> w(static_cast<size_t>(3) * (q + 1) * N);
  for (int c = 0; c < 3; ++c)
    for (int64_t j = 0; j < N; ++j) {
      const double x = u_soa[c * N + j];
      for (int a = 0; a <= q; ++a) {
        double num = 1.0, den = 1.0;
        for (int b = 0; b <= q; ++b)
          if (b != a) {
            num *= x - b;
            den *= a - b;
          }
        w[(static_cast<size_t>(c) * (q + 1) + a) * N + j] = num / den;
      }
    }
  return w;
}

// Stable counting sort of keys in [0, nkeys): order[] lists indices by key,
// start[k] = first position of key k (start[nkeys] = count).
void counting_sort(const std::vector<int64_t>& key, int64_t nkeys, std::vector<int32_t>& order,
                   std::vector<int32_t>& start) {
  start.assign(nkeys + 1, 0);
  for (int64_t k : key) start[k + 1]++;
  for (int64_t k = 0; k < nkeys; ++k) start[k + 1] += start[k];
  std::vector<int32_t> fill(start.begin(), start.end() - 1);
  order.resize(key.size());
  for (size_t i = 0; i < key.size(); ++i) order[fill[key[i]]++] = static_cast<int32_t>(i);
}

int planes_for(const fftpim_plan_s* p, int nrhs) {
  return p->prm.value_type == FFTPIM_REAL ? (nrhs + 1) / 2 : nrhs;
}

// ---------------------------------------------------------------------------
// FFT pass descriptors for the pruned, zero-padded convolution (Step 2)
// ---------------------------------------------------------------------------

int lines_per_block(int M, size_t esize, int64_t cap) {
  int T = 1;
  while (static_cast<size_t>(T) * 2 * M * esize <= kLdsBudget && T * 2 <= cap) T *= 2;
  return T;
}

FftPassDesc pass_desc(int M, int n_in, int n_out, bool contig, int64_t nouter, int64_t ncols, int64_t in_line,
                      int64_t in_outer, int64_t out_line, int64_t out_outer, size_t esize) {
  FftPassDesc d{};
  d.M = M;
  d.logM = ilog2(M);
  d.n_in = n_in;
  d.n_out = n_out;
  d.contig = contig ? 1 : 0;
  d.nouter = nouter;
  d.ncols = contig ? 1 : ncols;
  d.in_line = in_line;
  d.in_col = 1;
  d.in_outer = in_outer;
  d.out_line = out_line;
  d.out_col = 1;
  d.out_outer = out_outer;
  d.T = contig ? lines_per_block(M, esize, 1 << 20) : lines_per_block(M, esize, ncols);
  d.spec_line = 0;
  d.spec_col = 0;
  d.spec_div = 1;
  return d;
}

// Zero-padded (aperiodic) 3D convolution of a grid [n0][n1][n2][P] with a
// kernel given by its spectrum hat ([M0][M1][M2], scaled by 1/(M0 M1 M2)):
// pruned forward passes z, y, then x with the spectrum multiply fused
// (conjugated for the adjoint), pruned inverse passes y, z.  Reads in, uses
// bufA ([n0][n1][M2][P]) and bufB ([n0][M1][M2][P]), writes out (may be in).
template <typename R>
void grid_convolution(const int n[3], const int M[3], void* const tw[3], const void* hat, const void* in,
                      void* bufA, void* bufB, void* out, int P, bool adjoint, hipStream_t st) {
  // grids are [x][y][z][P]: a pass along one axis sees outer x line x columns,
  // the columns being the axes after it together with the planes
  const int nx = n[0], ny = n[1], nz = n[2];
  const int Mx = M[0], My = M[1], Mz = M[2];
  const size_t es = sizeof(cplx<R>);
  const int64_t xy = static_cast<int64_t>(nx) * ny;
  // z: in [nx*ny][nz][P] -> bufA [nx*ny][Mz][P]
  FftPassDesc dz = P == 1 ? pass_desc(Mz, nz, Mz, true, xy, 1, 1, nz, 1, Mz, es)
                          : pass_desc(Mz, nz, Mz, false, xy, P, P, static_cast<int64_t>(nz) * P, P,
                                      static_cast<int64_t>(Mz) * P, es);
  launch_fft_pass<R>(0, in, bufA, dz, tw[2], nullptr, false, st);
  // y: bufA [nx][ny][Mz*P] -> bufB [nx][My][Mz*P]
  const int64_t zc = static_cast<int64_t>(Mz) * P;
  FftPassDesc dy = pass_desc(My, ny, My, false, nx, zc, zc, ny * zc, zc, My * zc, es);
  launch_fft_pass<R>(0, bufA, bufB, dy, tw[1], nullptr, false, st);
  // x: in place on bufB [nx][My*Mz*P], fused spectrum multiply (one spectrum
  // value per (y, z) serves all planes)
  const int64_t cols = My * zc;
  FftPassDesc dx = pass_desc(Mx, nx, nx, false, 1, cols, cols, nx * cols, cols, nx * cols, es);
  dx.spec_line = static_cast<int64_t>(My) * Mz;
  dx.spec_col = 1;
  dx.spec_div = P;
  launch_fft_pass<R>(2, bufB, bufB, dx, tw[0], hat, adjoint, st);
  // inverse y: bufB [nx][My][Mz*P] -> bufA [nx][ny][Mz*P]
  FftPassDesc iy = pass_desc(My, My, ny, false, nx, zc, zc, My * zc, zc, ny * zc, es);
  launch_fft_pass<R>(1, bufB, bufA, iy, tw[1], nullptr, false, st);
  // inverse z: bufA [nx*ny][Mz][P] -> out [nx*ny][nz][P]
  FftPassDesc iz = P == 1 ? pass_desc(Mz, Mz, nz, true, xy, 1, 1, Mz, 1, nz, es)
                          : pass_desc(Mz, Mz, nz, false, xy, P, P, static_cast<int64_t>(Mz) * P, P,
                                      static_cast<int64_t>(nz) * P, es);
  launch_fft_pass<R>(1, bufA, out, iz, tw[2], nullptr, false, st);
}

// Near Step 2 (Sec. 3.3): in place on the work set's near grid.
template <typename R>
void near_convolution(fftpim_plan_s* p, const WorkSet& ws, int P, bool adjoint, hipStream_t st) {
  grid_convolution<R>(p->ng.n, p->M, p->twiddle, p->near_hat, ws.grid0, ws.bufA, ws.bufB, ws.grid0, P, adjoint, st);
}

SymArgs sym_args(const fftpim_plan_s* p) {
  SymArgs a{};
  const SymDev& d = p->symd;
  a.N = p->N;
  for (int c = 0; c < 3; ++c) a.nb[c] = p->nb[c];
  const CorrRegion reg = corr_region(p);
  a.R = std::max(reg.reach[0], std::max(reg.reach[1], reg.reach[2])) + p->ng.q;
  a.W = 2 * a.R + 1;
  a.k0 = p->lat.k0.real();
  a.k0_im = p->lat.k0.imag();
  a.max_box = d.max_box;
  a.npairs = d.npairs;
  a.nitems = d.nitems;
  a.nebox = d.nebox;
  a.box_start = p->box_start;
  a.ebox = d.ebox;
  a.pair_ebox_o = d.pair_ebox_o;
  a.pair_ebox_s = d.pair_ebox_s;
  a.pair_voff = d.pair_voff;
  a.pair_stride = d.pair_stride;
  a.groups = d.groups;
  a.item_order = d.item_order;
  a.item_ebox = d.item_ebox;
  a.item_gbeg = d.item_gbeg;
  a.item_yoff = d.item_yoff;
  a.ebox_item_beg = d.ebox_item_beg;
  a.in_ptr = d.in_ptr;
  a.in_base = d.in_base;
  return a;
}

GridArgs grid_args(const GridGeom& g) {
  GridArgs a{};
  for (int c = 0; c < 3; ++c) {
    a.n[c] = g.n[c];
    a.nint[c] = g.nint[c];
    a.nb[c] = g.nint[c] + 1;
  }
  return a;
}

FarArgs far_args(const fftpim_plan_s* p) {
  FarArgs f{};
  for (int c = 0; c < 3; ++c) {
    f.nf[c] = p->fg.n[c];
    f.nint[c] = p->fg.nint[c];
    f.nb[c] = p->fg.nint[c] + 1;
  }
  f.Ngf = static_cast<int64_t>(f.nf[0]) * f.nf[1] * f.nf[2];
  f.nboxes = static_cast<int64_t>(f.nb[0]) * f.nb[1] * f.nb[2];
  return f;
}

// Event pair around one stage when timing is on (pool grows on demand; the
// pairs are resolved by fftpim_stage_times).
struct StageTimer {
  fftpim_plan_s* p;
  hipStream_t st;
  int stage;
  size_t start = 0;
  bool on = false;
  StageTimer(fftpim_plan_s* p_, hipStream_t st_, int stage_) : p(p_), st(st_), stage(stage_) {
    if (!p->timing) return;
    while (p->ev_pool.size() < p->ev_used + 2) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      p->ev_pool.push_back(e);
    }
    start = p->ev_used;
    p->ev_used += 2;
    on = hipEventRecord(p->ev_pool[start], st) == hipSuccess;
  }
  ~StageTimer() {
    if (!on) return;
    if (hipEventRecord(p->ev_pool[start + 1], st) == hipSuccess) p->ev_pairs.emplace_back(stage, start);
  }
};

void resolve_timers(fftpim_plan_s* p) {
  for (auto& pr : p->ev_pairs) {
    float ms = 0.f;
    if (hipEventSynchronize(p->ev_pool[pr.second + 1]) == hipSuccess &&
        hipEventElapsedTime(&ms, p->ev_pool[pr.second], p->ev_pool[pr.second + 1]) == hipSuccess) {
      p->stage_ms[pr.first] += ms;
      p->stage_calls[pr.first] += 1;
    }
  }
  p->ev_pairs.clear();
  p->ev_used = 0;
}

// Step 4 of Sec. 3.3 (the correction) for one input, on stream sc.
template <typename R>
void correction_zone(fftpim_plan_s* p, bool adjoint, const void* in, int P, void* out, hipStream_t sc) {
  const int64_t N = p->N;
  if (p->sep) {
    // separate observers: observer rows forward, source rows (C^H) for the
    // conjugate transpose
    if (adjoint)
      launch_corr_spmv<R>(p->complex_kernel, p->rowptr_a, p->col_a, p->val_a, N, p->corr_order_a, p->corr_slots_a,
                          in, P, out, false, sc);
    else
      launch_corr_spmv<R>(p->complex_kernel, p->rowptr, p->col, p->val, p->No, p->corr_order, p->corr_slots, in, P,
                          out, false, sc);
    return;
  }
  const void* v = (adjoint && p->nonhermitian) ? p->val_adj : p->val;
  if (p->tile) {
    // real correction values: the operator is symmetric, so the conjugate
    // transpose uses the same tiles
    launch_corr_tile<R>(p->tile_rows, p->ntiles, p->tile_coff, p->tile_cols, p->tile_voff, p->tile_vals, in, P, out, sc);
  } else if (p->sym) {
    // in-cell part: A^H of a complex-symmetric block is conj(X conj(v))
    launch_sym_apply<R>(p->complex_kernel, sym_args(p), p->sym_vals, in, nullptr, P, P, adjoint, false, p->sym_ypart,
                        p->sym_zpart, out, nullptr, false, sc);
    if (p->nnz > 0)
      launch_corr_spmv<R>(p->complex_kernel, p->rowptr, p->col, v, N, p->corr_order, p->corr_slots, in, P, out, true,
                          sc);
  } else {
    launch_corr_spmv<R>(p->complex_kernel, p->rowptr, p->col, v, N, p->corr_order, p->corr_slots, in, P, out, false,
                        sc);
  }
}

// Steps 1-3 of Sec. 3.2 for one input, on stream sf.  The adjoint projects
// with the observer-grid weights, applies K^H and interpolates from the
// source grid.
// Far Steps 1-2 (Sec. 3.2): projection onto the source grid (observer grid
// for the adjoint) and the grid sum with K (K^H); the result is in ws.far_u.
template <typename R>
int far_field(fftpim_plan_s* p, const WorkSet& ws, bool adjoint, const void* in, int P, hipStream_t sf) {
  const int64_t N = adjoint ? p->No : p->N;  // points projected: observers for the adjoint
  const FarArgs fa = far_args(p);
  const int qf = p->fg.q;
  const int32_t* fbs = adjoint ? p->fbox_start_o : p->fbox_start_s;
  const int32_t* fpm = adjoint ? p->fperm_o : p->fperm_s;
  const double* fw_in = adjoint ? p->fo_w : p->fs_w;
  CHK(launch_far_moments<R>(qf, fa, fbs, fpm, fw_in, N, in, P, ws.far_mom, sf));
  CHK(launch_far_gather<R>(qf, fa, ws.far_mom, P, ws.far_q, sf));
  if (p->far_fft) {
    grid_convolution<R>(p->fg.n, p->Mf, p->ftwiddle, p->far_hat, ws.far_q, ws.far_bufA, ws.far_bufB, ws.far_u, P,
                        adjoint, sf);
    return FFTPIM_OK;
  }
  launch_far_apply<R>(fa, p->far_table, ws.far_q, ws.far_u, ws.far_part, P, adjoint,
                      p->prm.precision == FFTPIM_F32_FARBF16 ? 1 : (p->prm.precision == FFTPIM_F32_FARBF16X3 ? 2 : 0),
                      sf);
  return FFTPIM_OK;
}

template <typename R>
int far_zone(fftpim_plan_s* p, const WorkSet& ws, bool adjoint, const void* in, int P, void* out,
             hipStream_t sf) {
  const int64_t N = adjoint ? p->N : p->No;  // points interpolated: observers forward
  const FarArgs fa = far_args(p);
  const int qf = p->fg.q;
  const int32_t* fs_out = adjoint ? p->fs_s : p->fo_s;
  const double* fw_out = adjoint ? p->fs_w : p->fo_w;
  CHK(far_field<R>(p, ws, adjoint, in, P, sf));
  // interpolation side: observer-grid boxes (forward) or source-grid boxes (adjoint)
  const int32_t* fbs_out = adjoint ? p->fbox_start_s : p->fbox_start_o;
  const int32_t* fpm_out = adjoint ? p->fperm_s : p->fperm_o;
  const int maxb_out = adjoint ? p->fmax_box_s : p->fmax_box_o;
  if (!launch_far_interp_box<R>(qf, fa, fbs_out, fpm_out, maxb_out, fs_out, fw_out, N, ws.far_u, P, out, false, sf))
    CHK(launch_interp<R>(qf, grid_args(p->fg), fs_out, fw_out, N, ws.far_u, P, out, false, sf));
  return FFTPIM_OK;
}

// Steps 1-3 of Sec. 3.3 for one input, on stream sn (the same grid serves
// sources and observers).
// Near Steps 1-2 (Sec. 3.3): projection and the zero-padded FFT convolution
// (with conj(G^hat) for the adjoint); the result is in ws.grid0.
template <typename R>
int near_field(fftpim_plan_s* p, const WorkSet& ws, bool adjoint, const void* in, int P, hipStream_t sn) {
  const GridArgs ga = grid_args(p->ng);
  {
    StageTimer t(p, sn, FFTPIM_STAGE_NEAR_SPREAD);
    // the projected points: sources forward, observers for the adjoint
    // (the same set unless the plan has separate observers)
    if (p->wt_row != nullptr)
      launch_spread_csr<R>(p->wt_node, p->wt_nnodes, p->wt_row, p->wt_idx, p->wt_val,
                           static_cast<int64_t>(p->ng.n[0]) * p->ng.n[1] * p->ng.n[2], in, P, ws.grid0, sn);
    else if (adjoint)
      CHK(launch_spread_near<R>(p->ng.q, ga, p->box_start_o, p->near_s_o, p->near_w_o, p->No, in, P, ws.grid0, sn));
    else
      CHK(launch_spread_near<R>(p->ng.q, ga, p->box_start, p->near_s, p->near_w, p->N, in, P, ws.grid0, sn));
  }
  {
    StageTimer t(p, sn, FFTPIM_STAGE_NEAR_FFT);
    near_convolution<R>(p, ws, P, adjoint, sn);
  }
  return FFTPIM_OK;
}

template <typename R>
int near_grid_zone(fftpim_plan_s* p, const WorkSet& ws, bool adjoint, const void* in, int P, void* out,
                   hipStream_t sn) {
  const GridArgs ga = grid_args(p->ng);
  CHK(near_field<R>(p, ws, adjoint, in, P, sn));
  {
    StageTimer t(p, sn, FFTPIM_STAGE_NEAR_INTERP);
    if (adjoint)
      CHK(launch_interp<R>(p->ng.q, ga, p->near_s, p->near_w, p->N, ws.grid0, P, out, false, sn));
    else
      CHK(launch_interp<R>(p->ng.q, ga, p->near_s_o, p->near_w_o, p->No, ws.grid0, P, out, false, sn));
  }
  return FFTPIM_OK;
}

// The "exclude self" option (Eq. (5) read literally, n != m): the apply
// subtracts C_self q_m, C_self = lim_{r->0}[G^p(r) - G0(r)], and its
// conjugate transpose conj(C_self) v_m.
DiagTerm self_term(const fftpim_plan_s* p, const void* packed_in, bool adjoint) {
  DiagTerm d;
  if (p->prm.self_mode != FFTPIM_SELF_EXCLUDE) return d;
  d.in = packed_in;
  d.re = -p->self_coef.real();
  d.im = adjoint ? p->self_coef.imag() : -p->self_coef.imag();
  return d;
}

template <typename R>
int run_apply(fftpim_plan_s* p, int parts, bool adjoint, const void* in, void* out, int nrhs, hipStream_t st,
              bool finalize) {
  // the input lives on the sources (observers for the adjoint), the output
  // on the observers (sources); one set unless the plan has separate observers
  const int64_t N = adjoint ? p->No : p->N;
  const int64_t Nout = adjoint ? p->N : p->No;
  const int32_t* perm_in = adjoint ? p->perm_o : p->perm;
  const int32_t* perm_out = adjoint ? p->perm : p->perm_o;
  const int P = planes_for(p, nrhs);
  const bool real_io = p->prm.value_type == FFTPIM_REAL;
  const bool use_perm = p->prm.order_io == FFTPIM_ORDER_USER;
  p->last_stream = st;
  if (p->timing && p->ev_used > 4096) resolve_timers(p);
  {
    StageTimer t(p, st, FFTPIM_STAGE_PACK);
    launch_pack<R>(in, p->q_int, perm_in, N, nrhs, P, real_io, use_perm, st);
    if (finalize && !adjoint && p->lat.npsp()) {
      launch_plane_sums<R>(p->q_int, nullptr, nullptr, N, P, p->sums_work, p->sums, st);
      launch_check_neutral(p->sums, P, p->prm.precision != FFTPIM_F64 ? 1e-5 : 1e-10, p->status_dev, st);
    }
  }
  // Fork: the correction (Sec. 3.3 Step 4), the near-grid steps and the far
  // zone (Sec. 3.2) only read the packed amplitudes, so each runs on a stream
  // of the plan (the paper runs near and far zones concurrently on two
  // streams, Sec. 4.2) and the caller's stream joins them.  Each part writes
  // its own buffer; the unpack sums them in a fixed order.
  const bool do_corr = (parts & FFTPIM_PART_NEAR_CORR) != 0;
  const bool do_far = (parts & FFTPIM_PART_FAR) != 0;
  const bool do_near = (parts & FFTPIM_PART_NEAR_GRID) != 0;
  HIPCHK(hipEventRecord(p->ev_fork, st));
  if (do_corr) {
    hipStream_t sc = p->s_corr;
    HIPCHK(hipStreamWaitEvent(sc, p->ev_fork, 0));
    {
      StageTimer t(p, sc, FFTPIM_STAGE_NEAR_CORR);
      correction_zone<R>(p, adjoint, p->q_int, P, p->u_corr, sc);
    }
    HIPCHK(hipEventRecord(p->ev_corr, sc));
  }
  if (do_far) {
    hipStream_t sf = p->s_far;
    HIPCHK(hipStreamWaitEvent(sf, p->ev_fork, 0));
    {
      StageTimer t(p, sf, FFTPIM_STAGE_FAR);
      CHK(far_zone<R>(p, p->ws, adjoint, p->q_int, P, p->u_far, sf));
    }
    HIPCHK(hipEventRecord(p->ev_far, sf));
  }
  if (do_near) {
    hipStream_t sn = p->s_near;
    HIPCHK(hipStreamWaitEvent(sn, p->ev_fork, 0));
    CHK(near_grid_zone<R>(p, p->ws, adjoint, p->q_int, P, p->u_int, sn));
    HIPCHK(hipEventRecord(p->ev_near, sn));
  }
  // join
  if (do_corr) HIPCHK(hipStreamWaitEvent(st, p->ev_corr, 0));
  if (do_far) HIPCHK(hipStreamWaitEvent(st, p->ev_far, 0));
  if (do_near) HIPCHK(hipStreamWaitEvent(st, p->ev_near, 0));
  const void* un = do_near ? p->u_int : nullptr;
  const void* uc = do_corr ? p->u_corr : nullptr;
  const void* uf = do_far ? p->u_far : nullptr;
  const DiagTerm diag = self_term(p, p->q_int, adjoint);
  const double* mean = nullptr;
  if (finalize && adjoint && p->lat.npsp()) {
    // only the zero-mean part of A^H v is defined for the neutral static case
    launch_plane_sums<R>(un, uc, uf, Nout, P, p->sums_work, p->sums, st, diag);
    launch_mean_from_sums(p->sums, P, Nout, p->sums + 4 * p->nplanes_max, st);
    mean = p->sums + 4 * p->nplanes_max;
  }
  {
    StageTimer t(p, st, FFTPIM_STAGE_UNPACK);
    launch_unpack<R>(un, uc, uf, out, perm_out, Nout, nrhs, P, real_io, use_perm, mean, st, diag);
  }
  if (hipPeekAtLastError() != hipSuccess) return FFTPIM_ERR_DEVICE;
  return FFTPIM_OK;
}

// Byte sizes of the arrays of one near-grid + far-zone work set (for the
// plan's largest plane count), in WorkSet field order.
constexpr int kWorkArrays = 9;
void work_set_sizes(const fftpim_plan_s* p, size_t sz[kWorkArrays]) {
  const size_t P = static_cast<size_t>(p->nplanes_max);
  const size_t es = cbytes(p);
  const GridGeom& g = p->ng;
  const GridGeom& f = p->fg;
  const size_t K1 = static_cast<size_t>(f.q + 1);
  const size_t fboxes = static_cast<size_t>(p->fnb[0]) * p->fnb[1] * p->fnb[2];
  const size_t Ngf = static_cast<size_t>(f.n[0]) * f.n[1] * f.n[2];
  // the split count never exceeds min(64, ceil(Ngf / 256)) for any nrhs
  const size_t max_splits = std::min<size_t>(64, std::max<size_t>(1, (Ngf + 255) / 256));
  sz[0] = static_cast<size_t>(g.n[0]) * g.n[1] * g.n[2] * P * es;        // grid0
  sz[1] = static_cast<size_t>(g.n[0]) * g.n[1] * p->M[2] * P * es;       // bufA
  sz[2] = static_cast<size_t>(g.n[0]) * p->M[1] * p->M[2] * P * es;      // bufB
  sz[3] = fboxes * K1 * K1 * K1 * P * es;                                // far_mom
  sz[4] = Ngf * P * es;                                                  // far_q
  sz[5] = Ngf * P * es;                                                  // far_u
  sz[6] = p->far_fft ? 0 : max_splits * Ngf * P * es;                    // far_part
  sz[7] = p->far_fft ? static_cast<size_t>(f.n[0]) * f.n[1] * p->Mf[2] * P * es : 0;   // far_bufA
  sz[8] = p->far_fft ? static_cast<size_t>(f.n[0]) * p->Mf[1] * p->Mf[2] * P * es : 0;  // far_bufB
}

void** work_set_slots(WorkSet& ws, int k) {
  void** slots[kWorkArrays] = {&ws.grid0, &ws.bufA, &ws.bufB,     &ws.far_mom, &ws.far_q,
                               &ws.far_u, &ws.far_part, &ws.far_bufA, &ws.far_bufB};
  return slots[k];
}

int alloc_work_set(fftpim_plan_s* p, WorkSet& ws) {
  ws = WorkSet{};
  size_t sz[kWorkArrays];
  work_set_sizes(p, sz);
  for (int k = 0; k < kWorkArrays; ++k) {
    unsigned char* b = nullptr;
    CHK(dalloc(p, &b, sz[k]));
    *work_set_slots(ws, k) = b;
  }
  return FFTPIM_OK;
}

// Bytes of the fused pair's own arrays (a second work set, packed v and the
// three parts of w), each rounded up to 256 bytes as laid out by
// carve_pair_buffers.
size_t pair_buffer_bytes(const fftpim_plan_s* p) {
  size_t sz[kWorkArrays];
  work_set_sizes(p, sz);
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  size_t total = 0;
  for (int k = 0; k < kWorkArrays; ++k) total += up(sz[k]);
  total += 4 * up(static_cast<size_t>(p->N) * p->nplanes_max * cbytes(p));
  return total;
}

// Lays the fused pair's arrays out in one caller-provided device region of at
// least pair_buffer_bytes(p) bytes (256-byte aligned); allocates nothing.
PairBufs carve_pair_buffers(const fftpim_plan_s* p, unsigned char* base) {
  size_t sz[kWorkArrays];
  work_set_sizes(p, sz);
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  PairBufs pb;
  size_t off = 0;
  for (int k = 0; k < kWorkArrays; ++k) {
    *work_set_slots(pb.ws2, k) = base + off;
    off += up(sz[k]);
  }
  const size_t nb = up(static_cast<size_t>(p->N) * p->nplanes_max * cbytes(p));
  void** arr[4] = {&pb.v_int, &pb.u_int2, &pb.u_corr2, &pb.u_far2};
  for (int k = 0; k < 4; ++k) {
    *arr[k] = base + off;
    off += nb;
  }
  return pb;
}

// The fused pair's arrays owned by the plan, made on its first pair call.
int ensure_pair_buffers(fftpim_plan_s* p) {
  if (p->pair.v_int != nullptr) return FFTPIM_OK;
  // allocate into locals and publish only when every allocation succeeded; a
  // failure frees what this call made, so a retry starts from scratch
  PairBufs pb;
  int s = alloc_work_set(p, pb.ws2);
  const size_t bytes = static_cast<size_t>(p->N) * p->nplanes_max * cbytes(p);
  void** arr[4] = {&pb.v_int, &pb.u_int2, &pb.u_corr2, &pb.u_far2};
  for (int k = 0; k < 4 && s == FFTPIM_OK; ++k) {
    unsigned char* b = nullptr;
    s = dalloc(p, &b, bytes);
    *arr[k] = b;
  }
  if (s != FFTPIM_OK) {
    for (int k = 0; k < kWorkArrays; ++k) dfree(p, *work_set_slots(pb.ws2, k));
    for (int k = 0; k < 4; ++k) dfree(p, *arr[k]);
    return s;
  }
  p->pair = pb;
  return FFTPIM_OK;
}

// u = A q and w = A^H v in one pass.  The box-pair correction reads each
// stored block once for both products (its planes are q's followed by v's,
// the latter conjugated on the way in and out).  The near-grid and far-zone
// passes of the two products share two streams crosswise (near of A q then
// far of A^H v on one, far of A q then near of A^H v on the other), each
// product with its own work set, so both streams carry about the same work.
template <typename R>
int run_apply_pair(fftpim_plan_s* p, const PairBufs& pb, const void* q, void* u, const void* v, void* w, int nrhs,
                   hipStream_t st) {
  const int64_t N = p->N;
  const int P = planes_for(p, nrhs);
  const bool real_io = p->prm.value_type == FFTPIM_REAL;
  const bool use_perm = p->prm.order_io == FFTPIM_ORDER_USER;
  p->last_stream = st;
  if (p->timing && p->ev_used > 4096) resolve_timers(p);
  {
    StageTimer t(p, st, FFTPIM_STAGE_PACK);
    launch_pack<R>(q, p->q_int, p->perm, N, nrhs, P, real_io, use_perm, st);
    launch_pack<R>(v, pb.v_int, p->perm, N, nrhs, P, real_io, use_perm, st);
    if (p->lat.npsp()) {
      launch_plane_sums<R>(p->q_int, nullptr, nullptr, N, P, p->sums_work, p->sums, st);
      launch_check_neutral(p->sums, P, p->prm.precision != FFTPIM_F64 ? 1e-5 : 1e-10, p->status_dev, st);
    }
  }
  HIPCHK(hipEventRecord(p->ev_fork, st));
  {
    hipStream_t sc = p->s_corr;
    HIPCHK(hipStreamWaitEvent(sc, p->ev_fork, 0));
    {
      StageTimer t(p, sc, FFTPIM_STAGE_NEAR_CORR);
      // the fused box-pair pass stages both inputs in LDS (at most 64 KB, as
      // the single apply)
      if (p->sym && static_cast<int64_t>(p->symd.max_box) * 2 * P <= 2048) {
        launch_sym_apply<R>(p->complex_kernel, sym_args(p), p->sym_vals, p->q_int, pb.v_int, P, 2 * P, false, true,
                            p->sym_ypart, p->sym_zpart, p->u_corr, pb.u_corr2, false, sc);
        if (p->nnz > 0) {
          launch_corr_spmv<R>(p->complex_kernel, p->rowptr, p->col, p->val, N, p->corr_order, p->corr_slots, p->q_int,
                              P, p->u_corr, true, sc);
          launch_corr_spmv<R>(p->complex_kernel, p->rowptr, p->col, p->nonhermitian ? p->val_adj : p->val, N,
                              p->corr_order, p->corr_slots, pb.v_int, P, pb.u_corr2, true, sc);
        }
      } else {
        correction_zone<R>(p, false, p->q_int, P, p->u_corr, sc);
        correction_zone<R>(p, true, pb.v_int, P, pb.u_corr2, sc);
      }
    }
    HIPCHK(hipEventRecord(p->ev_corr, sc));
  }
  {
    hipStream_t sf = p->s_far;
    HIPCHK(hipStreamWaitEvent(sf, p->ev_fork, 0));
    {
      StageTimer t(p, sf, FFTPIM_STAGE_FAR);
      CHK(far_zone<R>(p, p->ws, false, p->q_int, P, p->u_far, sf));
    }
    CHK(near_grid_zone<R>(p, pb.ws2, true, pb.v_int, P, pb.u_int2, sf));
    HIPCHK(hipEventRecord(p->ev_far, sf));
  }
  {
    hipStream_t sn = p->s_near;
    HIPCHK(hipStreamWaitEvent(sn, p->ev_fork, 0));
    CHK(near_grid_zone<R>(p, p->ws, false, p->q_int, P, p->u_int, sn));
    {
      StageTimer t(p, sn, FFTPIM_STAGE_FAR);
      CHK(far_zone<R>(p, pb.ws2, true, pb.v_int, P, pb.u_far2, sn));
    }
    HIPCHK(hipEventRecord(p->ev_near, sn));
  }
  HIPCHK(hipStreamWaitEvent(st, p->ev_corr, 0));
  HIPCHK(hipStreamWaitEvent(st, p->ev_far, 0));
  HIPCHK(hipStreamWaitEvent(st, p->ev_near, 0));
  const DiagTerm diag_u = self_term(p, p->q_int, false), diag_w = self_term(p, pb.v_int, true);
  const double* mean = nullptr;
  if (p->lat.npsp()) {
    launch_plane_sums<R>(pb.u_int2, pb.u_corr2, pb.u_far2, N, P, p->sums_work, p->sums, st, diag_w);
    launch_mean_from_sums(p->sums, P, N, p->sums + 4 * p->nplanes_max, st);
    mean = p->sums + 4 * p->nplanes_max;
  }
  {
    StageTimer t(p, st, FFTPIM_STAGE_UNPACK);
    launch_unpack<R>(p->u_int, p->u_corr, p->u_far, u, p->perm, N, nrhs, P, real_io, use_perm, nullptr, st, diag_u);
    launch_unpack<R>(pb.u_int2, pb.u_corr2, pb.u_far2, w, p->perm, N, nrhs, P, real_io, use_perm, mean, st, diag_w);
  }
  if (hipPeekAtLastError() != hipSuccess) return FFTPIM_ERR_DEVICE;
  return FFTPIM_OK;
}

// Position gradient (see kernels_grad.hip): the forward near and far fields of
// q and the conjugate-transposed ones of g, differentiated interpolation at
// every point, and the correction entries differentiated on the fly.  All
// on the caller's stream; the [N][3] accumulator is added to in a fixed
// kernel order.
template <typename R>
int run_grad(fftpim_plan_s* p, const void* q, const void* g, int nrhs, double* grad, hipStream_t st) {
  const int64_t N = p->N;
  const int P = planes_for(p, nrhs);
  const bool real_io = p->prm.value_type == FFTPIM_REAL;
  const bool use_perm = p->prm.order_io == FFTPIM_ORDER_USER;
  CHK(ensure_pair_buffers(p));
  if (p->grad_acc == nullptr) CHK(dalloc(p, &p->grad_acc, static_cast<size_t>(N) * 3));
  p->last_stream = st;
  const PairBufs& pb = p->pair;
  launch_pack<R>(q, p->q_int, p->perm, N, nrhs, P, real_io, use_perm, st);
  launch_pack<R>(g, pb.v_int, p->perm, N, nrhs, P, real_io, use_perm, st);
  HIPCHK(hipMemsetAsync(p->grad_acc, 0, static_cast<size_t>(N) * 3 * sizeof(double), st));
  const GridArgs ga = grid_args(p->ng), fa = grid_args(p->fg);
  // near grid: forward field of q, adjoint field of g
  CHK(near_field<R>(p, p->ws, false, p->q_int, P, st));
  CHK(launch_interp_grad<R>(p->ng.q, ga, p->ng.h, p->near_s, p->near_u, N, p->ws.grid0, P, pb.v_int, p->grad_acc, st));
  CHK(near_field<R>(p, pb.ws2, true, pb.v_int, P, st));
  CHK(launch_interp_grad<R>(p->ng.q, ga, p->ng.h, p->near_s, p->near_u, N, pb.ws2.grid0, P, p->q_int, p->grad_acc,
                            st));
  // far zone: observer-grid weights on K W_s q, source-grid weights on K^H W_o g
  CHK(far_field<R>(p, p->ws, false, p->q_int, P, st));
  CHK(launch_interp_grad<R>(p->fg.q, fa, p->fg.h, p->fo_s, p->fo_u, N, p->ws.far_u, P, pb.v_int, p->grad_acc, st));
  CHK(far_field<R>(p, pb.ws2, true, pb.v_int, P, st));
  CHK(launch_interp_grad<R>(p->fg.q, fa, p->fg.h, p->fs_s, p->fs_u, N, pb.ws2.far_u, P, p->q_int, p->grad_acc, st));
  // correction entries of Eq. (er)
  CHK(launch_corr_grad(p->ng.q, p->complex_kernel, p->grad_ca, p->near_s, p->near_u, p->ng.h, p->pos3, p->box_start,
                       p->g0tab, P, p->q_int, pb.v_int, sizeof(R) == 4, p->grad_acc, st));
  launch_unpermute3(p->grad_acc, p->perm, N, use_perm, grad, st);
  if (hipPeekAtLastError() != hipSuccess) return FFTPIM_ERR_DEVICE;
  return FFTPIM_OK;
}

int apply_common(fftpim_plan_t plan, int parts, int adjoint, const void* in, void* out, int nrhs,
                 fftpim_stream_t stream, bool finalize) {
  if (!plan || !in || !out) return FFTPIM_ERR_INVALID_ARG;
  if (nrhs < 1 || nrhs > plan->prm.nrhs_max) return FFTPIM_ERR_INVALID_ARG;
  if (parts < 0 || parts > FFTPIM_PART_ALL) return FFTPIM_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (plan->prm.precision != FFTPIM_F64)
    return run_apply<float>(plan, parts, adjoint != 0, in, out, nrhs, st, finalize);
  return run_apply<double>(plan, parts, adjoint != 0, in, out, nrhs, st, finalize);
}

// ---------------------------------------------------------------------------
// plan construction
// ---------------------------------------------------------------------------

int validate(const fftpim_problem_t* pr, const fftpim_params_t* pm) {
  if (pr->periodic_dims < 1 || pr->periodic_dims > 3) return FFTPIM_ERR_INVALID_ARG;
  for (int c = 0; c < pr->periodic_dims; ++c)
    if (!(pr->L[c] > 0.0) || !std::isfinite(pr->L[c])) return FFTPIM_ERR_INVALID_ARG;
  if (!std::isfinite(pr->k0) || pr->k0 < 0.0) return FFTPIM_ERR_INVALID_ARG;
  if (!std::isfinite(pr->k0_im) || pr->k0_im > 0.0) return FFTPIM_ERR_INVALID_ARG;
  for (int c = 0; c < 3; ++c)
    if (!std::isfinite(pr->kt[c]) || !std::isfinite(pr->kt_im[c])) return FFTPIM_ERR_INVALID_ARG;
  if (pm->near_order < 1 || pm->near_order > kMaxNearOrder) return FFTPIM_ERR_INVALID_ARG;
  if (pm->far_order < 1 || pm->far_order > kMaxFarOrder) return FFTPIM_ERR_INVALID_ARG;
  for (int c = 0; c < 3; ++c) {
    if (pm->near_n[c] < pm->near_order + 2 || pm->near_n[c] > 2048) return FFTPIM_ERR_INVALID_ARG;
    if (pm->far_n[c] < pm->far_order + 2 || pm->far_n[c] > 512) return FFTPIM_ERR_INVALID_ARG;
  }
  if (!std::isfinite(pm->corr_ball) || pm->corr_ball < 0.0 || pm->corr_ball > kMaxCorrRadius)
    return FFTPIM_ERR_INVALID_ARG;
  if (pm->corr_ball == 0.0 && (pm->corr_radius < pm->near_order || pm->corr_radius > kMaxCorrRadius))
    return FFTPIM_ERR_INVALID_ARG;
  if (pm->n_images < 0 || pm->n_images > 2) return FFTPIM_ERR_INVALID_ARG;
  if (pm->far_sum < FFTPIM_FAR_AUTO || pm->far_sum > FFTPIM_FAR_FFT) return FFTPIM_ERR_INVALID_ARG;
  if (pm->far_sum == FFTPIM_FAR_FFT &&
      (pm->precision == FFTPIM_F32_FARBF16 || pm->precision == FFTPIM_F32_FARBF16X3))
    return FFTPIM_ERR_INVALID_ARG;
  if (pm->precision < FFTPIM_F64 || pm->precision > FFTPIM_F32_FARBF16X3) return FFTPIM_ERR_INVALID_ARG;
  if (pm->value_type != FFTPIM_REAL && pm->value_type != FFTPIM_COMPLEX) return FFTPIM_ERR_INVALID_ARG;
  if (pm->self_mode != FFTPIM_SELF_IMAGES && pm->self_mode != FFTPIM_SELF_EXCLUDE) return FFTPIM_ERR_INVALID_ARG;
  if (pm->order_io != FFTPIM_ORDER_USER && pm->order_io != FFTPIM_ORDER_PLAN) return FFTPIM_ERR_INVALID_ARG;
  if (pm->nrhs_max < 1 || pm->nrhs_max > 4096) return FFTPIM_ERR_INVALID_ARG;
  if (pm->corr_layout < FFTPIM_CORR_AUTO || pm->corr_layout > FFTPIM_CORR_TILE) return FFTPIM_ERR_INVALID_ARG;
  return FFTPIM_OK;
}

template <typename R>
std::vector<cplx<R>> twiddles(int M) {
  std::vector<cplx<R>> t(std::max(1, M / 2));
  for (int k = 0; k < M / 2; ++k) {
    double a = 2.0 * kPi * k / M;
    t[k] = cmake<R>(static_cast<R>(std::cos(a)), static_cast<R>(-std::sin(a)));
  }
  return t;
}

template <typename R>
int build_tables(fftpim_plan_s* p, hipStream_t st) {
  // twiddles per axis (working precision)
  for (int c = 0; c < 3; ++c) {
    cplx<R>* tw = nullptr;
    CHK(upload(p, &tw, twiddles<R>(p->M[c])));
    p->twiddle[c] = tw;
  }
  // near-zone table G^p_near at node offsets, zero padded, FFT in FP64
  const int dims = p->lat.dims;
  const int id = p->prm.n_images;
  std::vector<int> img;
  std::vector<double> ph;
  int lim[3];
  for (int c = 0; c < 3; ++c) lim[c] = c < dims ? id : 0;
  for (int ix = -lim[0]; ix <= lim[0]; ++ix)
    for (int iy = -lim[1]; iy <= lim[1]; ++iy)
      for (int iz = -lim[2]; iz <= lim[2]; ++iz) {
        img.push_back(ix);
        img.push_back(iy);
        img.push_back(iz);
        const cd f = p->lat.phase(ix, iy, iz);
        ph.push_back(f.real());
        ph.push_back(f.imag());
      }
  int* dimg = nullptr;
  double* dph = nullptr;
  CHK(upload(p, &dimg, img));
  CHK(upload(p, &dph, ph));
  NearTableArgs na{};
  for (int c = 0; c < 3; ++c) {
    na.M[c] = p->M[c];
    na.n[c] = p->ng.n[c];
    na.nint[c] = p->ng.nint[c];
    na.h[c] = p->ng.h[c];
  }
  na.k0 = p->lat.k0.real();
  na.k0_im = p->lat.k0.imag();
  na.nimg = static_cast<int>(img.size() / 3);
  na.img = dimg;
  na.phase = dph;
  const int64_t total = static_cast<int64_t>(p->M[0]) * p->M[1] * p->M[2];
  cplx<double>* T = nullptr;
  CHK(dalloc(p, &T, total));
  launch_near_table(T, na, st);
  cplx<double>* tw64[3];
  for (int c = 0; c < 3; ++c) CHK(upload(p, &tw64[c], twiddles<double>(p->M[c])));
  {
    const int Mx = p->M[0], My = p->M[1], Mz = p->M[2];
    const size_t es = sizeof(cplx<double>);
    FftPassDesc dz = pass_desc(Mz, Mz, Mz, true, static_cast<int64_t>(Mx) * My, 1, 1, Mz, 1, Mz, es);
    launch_fft_pass<double>(0, T, T, dz, tw64[2], nullptr, false, st);
    FftPassDesc dy = pass_desc(My, My, My, false, Mx, Mz, Mz, static_cast<int64_t>(My) * Mz, Mz,
                               static_cast<int64_t>(My) * Mz, es);
    launch_fft_pass<double>(0, T, T, dy, tw64[1], nullptr, false, st);
    const int64_t cols = static_cast<int64_t>(My) * Mz;
    FftPassDesc dx = pass_desc(Mx, Mx, Mx, false, 1, cols, cols, Mx * cols, cols, Mx * cols, es);
    launch_fft_pass<double>(0, T, T, dx, tw64[0], nullptr, false, st);
  }
  cplx<R>* hat = nullptr;
  CHK(dalloc(p, &hat, total));
  launch_scale_convert<R>(T, hat, total, 1.0 / static_cast<double>(total), st);
  p->near_hat = hat;
  HIPCHK(hipStreamSynchronize(st));
  dfree(p, T);
  for (int c = 0; c < 3; ++c) dfree(p, tw64[c]);
  dfree(p, dimg);
  dfree(p, dph);

  // far-zone table G^p_far at the offsets between observer and source grids,
  // evaluated on the device in FP64 (Sec. 3.2)
  std::vector<cd> ft;
  int nf[3] = {p->fg.n[0], p->fg.n[1], p->fg.n[2]};
  {
    FarTableArgs ta{};
    ta.dims = p->lat.dims;
    for (int c = 0; c < 3; ++c) {
      ta.nf[c] = nf[c];
      ta.delta[c] = p->fg.h[c];
      ta.L[c] = p->lat.L[c];
      ta.kt[c] = p->lat.kt[c].real();
      ta.kt_im[c] = p->lat.kt[c].imag();
    }
    ta.k0 = p->lat.k0.real();
    ta.k0_im = p->lat.k0.imag();
    ta.id = id;
    const int64_t total = static_cast<int64_t>(2 * nf[0] - 1) * (2 * nf[1] - 1) * (2 * nf[2] - 1);
    cplx<double>* dt = nullptr;
    CHK(dalloc(p, &dt, static_cast<size_t>(total)));
    if (p->lat.dims == 2 && !p->lat.npsp())
      launch_far_table_pgf2(ta, dt, st);
    else
      CHK(launch_far_table(ta, p->lat.npsp(), dt, st));
    if (p->far_fft) {
      // the table as one period of a circulant, its FP64 spectrum scaled by
      // 1/(Mfx Mfy Mfz) and stored in the working precision
      const int Mx = p->Mf[0], My = p->Mf[1], Mz = p->Mf[2];
      const int64_t mt = static_cast<int64_t>(Mx) * My * Mz;
      cplx<double>* C = nullptr;
      CHK(dalloc(p, &C, static_cast<size_t>(mt)));
      launch_far_circulant(dt, nf, p->Mf, C, st);
      cplx<double>* tw64[3];
      for (int c = 0; c < 3; ++c) CHK(upload(p, &tw64[c], twiddles<double>(p->Mf[c])));
      const size_t es = sizeof(cplx<double>);
      FftPassDesc dz = pass_desc(Mz, Mz, Mz, true, static_cast<int64_t>(Mx) * My, 1, 1, Mz, 1, Mz, es);
      launch_fft_pass<double>(0, C, C, dz, tw64[2], nullptr, false, st);
      FftPassDesc dy = pass_desc(My, My, My, false, Mx, Mz, Mz, static_cast<int64_t>(My) * Mz, Mz,
                                 static_cast<int64_t>(My) * Mz, es);
      launch_fft_pass<double>(0, C, C, dy, tw64[1], nullptr, false, st);
      const int64_t cols = static_cast<int64_t>(My) * Mz;
      FftPassDesc dx = pass_desc(Mx, Mx, Mx, false, 1, cols, cols, Mx * cols, cols, Mx * cols, es);
      launch_fft_pass<double>(0, C, C, dx, tw64[0], nullptr, false, st);
      cplx<R>* fh = nullptr;
      CHK(dalloc(p, &fh, static_cast<size_t>(mt)));
      launch_scale_convert<R>(C, fh, mt, 1.0 / static_cast<double>(mt), st);
      HIPCHK(hipStreamSynchronize(st));
      HIPCHK(hipGetLastError());
      // a non-finite table value (a series that failed) poisons the spectrum
      std::vector<cplx<double>> probe(static_cast<size_t>(total));
      HIPCHK(hipMemcpy(probe.data(), dt, total * sizeof(cplx<double>), hipMemcpyDeviceToHost));
      for (const auto& v : probe)
        if (!std::isfinite(v.x) || !std::isfinite(v.y)) return FFTPIM_ERR_UNSUPPORTED;
      dfree(p, C);
      dfree(p, dt);
      for (int c = 0; c < 3; ++c) dfree(p, tw64[c]);
      p->far_hat = fh;
      for (int c = 0; c < 3; ++c) {
        cplx<R>* tw = nullptr;
        CHK(upload(p, &tw, twiddles<R>(p->Mf[c])));
        p->ftwiddle[c] = tw;
      }
      return FFTPIM_OK;
    }
    std::vector<cplx<double>> ht(static_cast<size_t>(total));
    HIPCHK(hipMemcpyAsync(ht.data(), dt, total * sizeof(cplx<double>), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipGetLastError());
    dfree(p, dt);
    ft.resize(static_cast<size_t>(total));
    for (int64_t i = 0; i < total; ++i) ft[i] = cd(ht[i].x, ht[i].y);
  }
  std::vector<cplx<R>> ftr(ft.size());
  for (size_t i = 0; i < ft.size(); ++i) {
    if (!std::isfinite(ft[i].real()) || !std::isfinite(ft[i].imag())) return FFTPIM_ERR_UNSUPPORTED;
    ftr[i] = cmake<R>(static_cast<R>(ft[i].real()), static_cast<R>(ft[i].imag()));
  }
  cplx<R>* dft = nullptr;
  CHK(upload(p, &dft, ftr));
  p->far_table = dft;
  return FFTPIM_OK;
}

// Symmetric in-cell blocks: pairs (B, B') of non-empty near-grid boxes with
// B <= B' (box id order) within r_c boxes (no image shift).  The pairs of a
// box are cut into lane groups (SymGroup) and the groups into work items of
// at most kGroupsPerItem groups; values are filled on the device.
constexpr int kGroupsPerItem = 12;
constexpr int kLanes = 64;
inline int64_t zround(int64_t n) { return (n + kSymZAlign - 1) / kSymZAlign * kSymZAlign; }

int build_sym(fftpim_plan_s* p, const std::vector<int32_t>& start, const double* pos3_dev, const void* g0tab,
              const CorrArgs& ca, hipStream_t st) {
  const int nbx = p->nb[0], nby = p->nb[1], nbz = p->nb[2];
  const int64_t nboxes = static_cast<int64_t>(nbx) * nby * nbz;
  const CorrRegion reg = corr_region(p);
  std::vector<int32_t> ebox, ebox_of_box(nboxes, -1);
  int max_box = 0;
  for (int64_t b = 0; b < nboxes; ++b) {
    const int cnt = start[b + 1] - start[b];
    if (cnt > 0) {
      ebox_of_box[b] = static_cast<int32_t>(ebox.size());
      ebox.push_back(static_cast<int32_t>(b));
      max_box = std::max(max_box, cnt);
    }
  }
  const int64_t E = static_cast<int64_t>(ebox.size());
  std::vector<int32_t> po, ps, item_ebox, ebox_item_beg(E + 1, 0);
  std::vector<int64_t> pvoff, pstride, item_gbeg, item_yoff;
  std::vector<SymGroup> groups;
  // senders of column partials to each box, in box order: (destination, slot)
  std::vector<std::vector<int64_t>> in_lists(E);
  int64_t voff = 0, zoff = 0, yoff = 0;
  std::vector<int64_t> gpairs;  // pairs of the open group
  bool layout_ok = true;
  // source point of column c of a group (the apply kernel's rule)
  auto col_point = [](const SymGroup& g, int c) {
    int n = g.n0[0] + c;
    if (c >= g.end[0]) n = g.n0[1] + c - g.end[0];
    if (c >= g.end[1]) n = g.n0[2] + c - g.end[1];
    if (c >= g.end[2]) n = g.n0[3] + c - g.end[2];
    return n;
  };
  for (int64_t k = 0; k < E; ++k) {
    const int64_t B = ebox[k];
    const int bz = static_cast<int>(B % nbz), by = static_cast<int>((B / nbz) % nby),
              bx = static_cast<int>(B / (static_cast<int64_t>(nbz) * nby));
    const int nB = start[B + 1] - start[B];
    const int64_t gfirst = static_cast<int64_t>(groups.size());
    SymGroup g{};
    int nseg = 0;
    auto open_group = [&]() {
      g = SymGroup{};
      g.voff = voff;
      g.zoff = zoff;
      for (int s = 0; s < 4; ++s) g.end[s] = kLanes;
      nseg = 0;
      gpairs.clear();
    };
    auto close_group = [&]() {
      if (g.cum == 0) return;
      g.stride = g.cum;
      int col = 0;
      for (int64_t j : gpairs) {
        pvoff[j] = g.voff + col;
        pstride[j] = g.cum;
        const int64_t Bp = ebox[ps[j]];
        const int nj = start[Bp + 1] - start[Bp];
        // the kernel's column -> point map must give this pair's points
        if (col_point(g, col) != start[Bp] || col_point(g, col + nj - 1) != start[Bp] + nj - 1) layout_ok = false;
        if (ps[j] != k) in_lists[ps[j]].push_back(g.zoff + col);
        col += nj;
      }
      if (col != g.cum || g.cum > kLanes) layout_ok = false;
      groups.push_back(g);
      voff += static_cast<int64_t>(nB) * g.cum;
      zoff += zround(g.cum);
    };
    open_group();
    for (int cx = std::max(0, bx - reg.reach[0]); cx <= std::min(nbx - 1, bx + reg.reach[0]); ++cx)
      for (int cy = std::max(0, by - reg.reach[1]); cy <= std::min(nby - 1, by + reg.reach[1]); ++cy)
        for (int cz = std::max(0, bz - reg.reach[2]); cz <= std::min(nbz - 1, bz + reg.reach[2]); ++cz) {
          const int64_t Bp = (static_cast<int64_t>(cx) * nby + cy) * nbz + cz;
          if (Bp < B || ebox_of_box[Bp] < 0) continue;
          if (reg.ball && !ball_close(reg.bw, reg.br2, bx - cx, by - cy, bz - cz)) continue;
          const int kp = ebox_of_box[Bp];
          const int n0 = start[Bp], nj = start[Bp + 1] - n0;
          const int64_t j = static_cast<int64_t>(po.size());
          po.push_back(static_cast<int32_t>(k));
          ps.push_back(kp);
          pvoff.push_back(0);
          pstride.push_back(0);
          if (nj > kLanes) {
            // a pair wider than the wavefront: its own block, cut into column chunks
            close_group();
            pvoff[j] = voff;
            pstride[j] = nj;
            if (kp != k) in_lists[kp].push_back(zoff);
            for (int c0 = 0; c0 < nj; c0 += kLanes) {
              SymGroup w{};
              w.voff = voff + c0;
              w.zoff = zoff + c0;
              w.cum = std::min(kLanes, nj - c0);
              w.stride = nj;
              w.n0[0] = n0 + c0;
              w.end[0] = w.cum;
              for (int s = 1; s < 4; ++s) w.end[s] = kLanes;
              if (kp == k) w.diag_hi = w.cum;
              groups.push_back(w);
            }
            voff += static_cast<int64_t>(nB) * nj;
            zoff += zround(nj);
            open_group();
            continue;
          }
          const bool contiguous = nseg > 0 && n0 == g.n0[nseg - 1] + (g.end[nseg - 1] - (nseg > 1 ? g.end[nseg - 2] : 0));
          if (g.cum + nj > kLanes || (!contiguous && nseg == 4)) {
            close_group();
            open_group();
          }
          const bool cont = nseg > 0 && n0 == g.n0[nseg - 1] + (g.end[nseg - 1] - (nseg > 1 ? g.end[nseg - 2] : 0));
          if (cont) {
            g.end[nseg - 1] += nj;
          } else {
            g.n0[nseg] = n0;
            g.end[nseg] = g.cum + nj;
            ++nseg;
          }
          if (kp == k) {
            g.diag_lo = g.cum;
            g.diag_hi = g.cum + nj;
          }
          g.cum += nj;
          gpairs.push_back(j);
        }
    close_group();
    const int64_t glast = static_cast<int64_t>(groups.size());
    ebox_item_beg[k] = static_cast<int32_t>(item_ebox.size());
    for (int64_t a0 = gfirst; a0 < glast; a0 += kGroupsPerItem) {
      item_ebox.push_back(static_cast<int32_t>(k));
      item_gbeg.push_back(a0);
      item_yoff.push_back(yoff);
      yoff += nB;
    }
  }
  ebox_item_beg[E] = static_cast<int32_t>(item_ebox.size());
  item_gbeg.push_back(static_cast<int64_t>(groups.size()));
  for (const SymGroup& g : groups)
    if (g.cum < 1 || g.cum > kLanes || g.diag_lo < 0 || g.diag_hi > g.cum || g.diag_lo > g.diag_hi ||
        col_point(g, 0) < 0 || col_point(g, g.cum - 1) >= p->N)
      layout_ok = false;
  if (!layout_ok) return FFTPIM_ERR_DEVICE;
  // launch order: items by decreasing number of values (largest first keeps
  // the tail of the launch short); ties by item index
  const int64_t nit = static_cast<int64_t>(item_ebox.size());
  std::vector<int64_t> cost(nit, 0);
  for (int64_t it = 0; it < nit; ++it) {
    const int64_t B = ebox[item_ebox[it]];
    const int64_t nB = start[B + 1] - start[B];
    for (int64_t gi = item_gbeg[it]; gi < item_gbeg[it + 1]; ++gi) cost[it] += nB * groups[gi].cum;
  }
  std::vector<int32_t> item_order(nit);
  for (int64_t it = 0; it < nit; ++it) item_order[it] = static_cast<int32_t>(it);
  std::stable_sort(item_order.begin(), item_order.end(), [&](int32_t x, int32_t y) { return cost[x] > cost[y]; });
  std::vector<int64_t> in_ptr(E + 1, 0), in_base;
  for (int64_t k = 0; k < E; ++k) in_ptr[k + 1] = in_ptr[k] + static_cast<int64_t>(in_lists[k].size());
  in_base.reserve(in_ptr[E]);
  for (int64_t k = 0; k < E; ++k) in_base.insert(in_base.end(), in_lists[k].begin(), in_lists[k].end());
  SymDev& d = p->symd;
  d.npairs = static_cast<int64_t>(po.size());
  d.nitems = static_cast<int64_t>(item_ebox.size());
  d.nebox = E;
  d.ngroups = static_cast<int64_t>(groups.size());
  d.yslots = yoff;
  d.zslots = zoff;
  d.max_box = max_box;
  CHK(upload(p, &d.ebox, ebox));
  CHK(upload(p, &d.pair_ebox_o, po));
  CHK(upload(p, &d.pair_ebox_s, ps));
  CHK(upload(p, &d.pair_voff, pvoff));
  CHK(upload(p, &d.pair_stride, pstride));
  CHK(upload(p, &d.groups, groups));
  CHK(upload(p, &d.item_ebox, item_ebox));
  CHK(upload(p, &d.item_order, item_order));
  CHK(upload(p, &d.item_gbeg, item_gbeg));
  CHK(upload(p, &d.item_yoff, item_yoff));
  CHK(upload(p, &d.ebox_item_beg, ebox_item_beg));
  CHK(upload(p, &d.in_ptr, in_ptr));
  CHK(upload(p, &d.in_base, in_base));
  p->sym_nvals = voff;
  unsigned char* v = nullptr;
  CHK(dalloc(p, &v, static_cast<size_t>(voff) * (p->complex_kernel ? 16 : 8)));
  p->sym_vals = v;
  SymArgs sa = sym_args(p);
  sa.R = ca.R;
  sa.W = ca.W;
  CHK(launch_sym_fill(p->ng.q, p->complex_kernel, sa, p->near_w, pos3_dev, g0tab, p->sym_vals, st));
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipGetLastError());
  if (std::getenv("FFTPIM_LOG"))
    std::fprintf(stderr, "fftpim plan: symmetric blocks: %lld boxes, %lld pairs, %lld groups, %lld values, max box %d\n",
                 static_cast<long long>(E), static_cast<long long>(d.npairs), static_cast<long long>(d.ngroups),
                 static_cast<long long>(voff), max_box);
  return FFTPIM_OK;
}

// Processing order of the CSR rows: tiles of kRowTile^3 near-grid boxes, each
// tile's rows handed to one XCD (workgroups are dispatched to the XCDs round
// robin, so slot block b runs on XCD b mod kXcds).  The rows of a tile share
// most of their correction columns, so their amplitude gathers hit that XCD's
// L2.  Tiles go, in tile order, to the least loaded XCD.
constexpr int kRowTile = 8, kXcds = 8, kRowsPerBlock = 4;

void build_row_order(const std::vector<int32_t>& start, const int nb[3], int64_t N, std::vector<int32_t>& order) {
  int nt[3];
  for (int c = 0; c < 3; ++c) nt[c] = (nb[c] + kRowTile - 1) / kRowTile;
  std::vector<std::vector<int32_t>> seq(kXcds);
  std::vector<int64_t> load(kXcds, 0);
  std::vector<int32_t> rows;
  for (int tx = 0; tx < nt[0]; ++tx)
    for (int ty = 0; ty < nt[1]; ++ty)
      for (int tz = 0; tz < nt[2]; ++tz) {
        rows.clear();
        for (int bx = tx * kRowTile; bx < std::min(nb[0], (tx + 1) * kRowTile); ++bx)
          for (int by = ty * kRowTile; by < std::min(nb[1], (ty + 1) * kRowTile); ++by)
            for (int bz = tz * kRowTile; bz < std::min(nb[2], (tz + 1) * kRowTile); ++bz) {
              const int64_t b = (static_cast<int64_t>(bx) * nb[1] + by) * nb[2] + bz;
              for (int32_t m = start[b]; m < start[b + 1]; ++m) rows.push_back(m);
            }
        if (rows.empty()) continue;
        const int x = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
        seq[x].insert(seq[x].end(), rows.begin(), rows.end());
        load[x] += static_cast<int64_t>(rows.size());
      }
  int64_t maxlen = 0;
  for (const auto& s : seq) maxlen = std::max<int64_t>(maxlen, static_cast<int64_t>(s.size()));
  const int64_t per_xcd = (maxlen + kRowsPerBlock - 1) / kRowsPerBlock;
  order.assign(static_cast<size_t>(per_xcd * kXcds * kRowsPerBlock), -1);
  for (int x = 0; x < kXcds; ++x)
    for (int64_t i = 0; i < static_cast<int64_t>(seq[x].size()); ++i) {
      const int64_t blk = (i / kRowsPerBlock) * kXcds + x;
      order[static_cast<size_t>(blk * kRowsPerBlock + i % kRowsPerBlock)] = seq[x][static_cast<size_t>(i)];
    }
  (void)N;
}

// Dense row tiles for real correction values.  Observers are ordered by the
// Morton key of their near-grid box (so 16 consecutive observers sit in a
// compact group of boxes and share most corrected sources) and cut into
// tiles of 16; a tile stores the 16 x C block over the union of its
// observers' CSR columns, zeros included, and the CSR is released.
constexpr int kTileRows = 16;

inline uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  uint64_t k = 0;
  for (int i = 0; i < 21; ++i)
    k |= (static_cast<uint64_t>((x >> i) & 1) << (3 * i + 2)) | (static_cast<uint64_t>((y >> i) & 1) << (3 * i + 1)) |
         (static_cast<uint64_t>((z >> i) & 1) << (3 * i));
  return k;
}

int build_tiles(fftpim_plan_s* p, const std::vector<int32_t>& start, const std::vector<int64_t>& rowptr,
                hipStream_t st) {
  const int64_t N = p->N;
  const int nbx = p->nb[0], nby = p->nb[1], nbz = p->nb[2];
  std::vector<uint64_t> key(N);
  for (int bx = 0; bx < nbx; ++bx)
    for (int by = 0; by < nby; ++by)
      for (int bz = 0; bz < nbz; ++bz) {
        const int64_t b = (static_cast<int64_t>(bx) * nby + by) * nbz + bz;
        const uint64_t k = morton3(bx, by, bz);
        for (int32_t m = start[b]; m < start[b + 1]; ++m) key[m] = k;
      }
  std::vector<int32_t> order(N);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return key[x] < key[y]; });
  const int64_t ntiles = (N + kTileRows - 1) / kTileRows;
  std::vector<int32_t> trows(static_cast<size_t>(ntiles * kTileRows), -1);
  std::copy(order.begin(), order.end(), trows.begin());
  // union of the CSR columns of each tile's observers (host threads)
  std::vector<int32_t> hcol(static_cast<size_t>(p->nnz));
  if (p->nnz > 0) HIPCHK(hipMemcpy(hcol.data(), p->col, p->nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
  std::vector<std::vector<int32_t>> tcols(ntiles);
  const int nth = static_cast<int>(std::max<unsigned>(1, std::min<unsigned>(16, std::thread::hardware_concurrency())));
  std::vector<std::thread> pool;
  for (int w = 0; w < nth; ++w)
    pool.emplace_back([&, w]() {
      std::vector<int64_t> seen(N, -1);
      for (int64_t t = w; t < ntiles; t += nth) {
        std::vector<int32_t>& out = tcols[t];
        for (int r = 0; r < kTileRows; ++r) {
          const int32_t m = trows[t * kTileRows + r];
          if (m < 0) continue;
          for (int64_t j = rowptr[m]; j < rowptr[m + 1]; ++j) {
            const int32_t n = hcol[j];
            if (seen[n] != t) {
              seen[n] = t;
              out.push_back(n);
            }
          }
        }
        std::sort(out.begin(), out.end());
      }
    });
  for (auto& th : pool) th.join();
  std::vector<int64_t> coff(ntiles + 1, 0), voff(ntiles + 1, 0);
  for (int64_t t = 0; t < ntiles; ++t) {
    const int64_t C = static_cast<int64_t>(tcols[t].size());
    coff[t + 1] = coff[t] + C;
    voff[t + 1] = voff[t] + 64 * ((C + 3) / 4);
  }
  std::vector<int32_t> cols(static_cast<size_t>(coff[ntiles]));
  for (int64_t t = 0; t < ntiles; ++t) std::copy(tcols[t].begin(), tcols[t].end(), cols.begin() + coff[t]);
  tcols.clear();
  CHK(upload(p, &p->tile_rows, trows));
  CHK(upload(p, &p->tile_coff, coff));
  CHK(upload(p, &p->tile_cols, cols));
  CHK(upload(p, &p->tile_voff, voff));
  CHK(dalloc(p, &p->tile_vals, static_cast<size_t>(voff[ntiles])));
  HIPCHK(hipMemsetAsync(p->tile_vals, 0, static_cast<size_t>(voff[ntiles]) * sizeof(double), st));
  launch_tile_fill(p->tile_rows, ntiles * kTileRows, p->rowptr, p->col, static_cast<const double*>(p->val),
                   p->tile_coff, p->tile_cols, p->tile_voff, p->tile_vals, st);
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipGetLastError());
  p->ntiles = ntiles;
  p->tile_nvals = voff[ntiles];
  // the tiles replace the CSR
  dfree(p, p->col);
  dfree(p, p->val);
  p->col = nullptr;
  p->val = nullptr;
  if (std::getenv("FFTPIM_LOG"))
    std::fprintf(stderr, "fftpim plan: row tiles: %lld tiles, %lld union columns, %lld values (CSR nnz %lld)\n",
                 static_cast<long long>(ntiles), static_cast<long long>(coff[ntiles]),
                 static_cast<long long>(voff[ntiles]), static_cast<long long>(p->nnz));
  return FFTPIM_OK;
}

// start: the source box sort; start_o, pos3_o: the observers' when they are
// a separate set (nullptr otherwise).
int build_correction(fftpim_plan_s* p, const std::vector<int32_t>& start, const double* pos3_dev,
                     const std::vector<int32_t>* start_o, const double* pos3_o, hipStream_t st) {
  const int q = p->ng.q, id = p->prm.n_images;
  const CorrRegion reg = corr_region(p);
  const int rc = std::max(reg.reach[0], std::max(reg.reach[1], reg.reach[2]));
  const int dims = p->lat.dims;
  const int A = 2 * id + 1;
  CorrArgs ca{};
  ca.ball = reg.ball;
  for (int c = 0; c < 3; ++c) ca.bw[c] = reg.bw[c];
  ca.br2 = reg.br2;
  for (int c = 0; c < 3; ++c) {
    ca.nb[c] = p->nb[c];
    ca.nint[c] = p->ng.nint[c];
    ca.per[c] = c < dims ? 1 : 0;
    ca.L[c] = p->lat.L[c];
  }
  ca.rc = rc;
  ca.id = id;
  ca.R = rc + q;
  ca.W = 2 * ca.R + 1;
  ca.N = p->N;
  ca.Nc = p->N;
  ca.k0 = p->lat.k0.real();
  ca.k0_im = p->lat.k0.imag();
  ca.nimg_axis = A;
  ca.images_only = p->sym ? 1 : 0;
  // image phases indexed by (gx, gy, gz), image g - id on periodic axes; the
  // conjugate-transpose values use conj(phase of image -i) (the same as the
  // phase of image i for a real phase shift)
  std::vector<double> ph(4 * A * A * A, 0.0);
  for (int gx = 0; gx < A; ++gx)
    for (int gy = 0; gy < A; ++gy)
      for (int gz = 0; gz < A; ++gz) {
        int im[3] = {gx - id * ca.per[0], gy - id * ca.per[1], gz - id * ca.per[2]};
        const cd f = p->lat.phase(im[0], im[1], im[2]);
        const cd fa = std::conj(p->lat.phase(-im[0], -im[1], -im[2]));
        int k = (gx * A + gy) * A + gz;
        ph[2 * k] = f.real();
        ph[2 * k + 1] = f.imag();
        ph[2 * A * A * A + 2 * k] = fa.real();
        ph[2 * A * A * A + 2 * k + 1] = fa.imag();
      }
  double* dph = nullptr;
  CHK(upload(p, &dph, ph));
  ca.phase = dph;
  ca.phase_adj = dph + 2 * A * A * A;
  // per-axis candidate source boxes for every observer box
  int32_t* doff[3];
  int32_t* dent[3];
  for (int c = 0; c < 3; ++c) {
    const int nint = p->ng.nint[c];
    const int rcc = reg.reach[c];
    std::vector<int32_t> off(nint + 2, 0), ent;
    for (int S = 0; S <= nint; ++S) {
      off[S] = static_cast<int32_t>(ent.size());
      for (int b = 0; b <= nint; ++b) {
        int mask = 0;
        if (ca.per[c]) {
          for (int i = -id; i <= id; ++i)
            if (std::abs(S - b - i * nint) <= rcc) mask |= 1 << (i + id);
        } else if (std::abs(S - b) <= rcc) {
          mask = 1;
        }
        if (mask) ent.push_back(b | (mask << 16));
      }
    }
    off[nint + 1] = static_cast<int32_t>(ent.size());
    CHK(upload(p, &doff[c], off));
    CHK(upload(p, &dent[c], ent));
    ca.loff[c] = doff[c];
    ca.lent[c] = dent[c];
  }
  // G0 at node offsets [-R, R]^3 (0 at the origin)
  const int W = ca.W, Rr = ca.R;
  std::vector<cplx<double>> g0t(static_cast<size_t>(W) * W * W);
  for (int ex = -Rr; ex <= Rr; ++ex)
    for (int ey = -Rr; ey <= Rr; ++ey)
      for (int ez = -Rr; ez <= Rr; ++ez) {
        size_t k = (static_cast<size_t>(ex + Rr) * W + (ey + Rr)) * W + (ez + Rr);
        if (ex == 0 && ey == 0 && ez == 0) {
          g0t[k] = cmake<double>(0.0, 0.0);
          continue;
        }
        double dx = ex * p->ng.h[0], dy = ey * p->ng.h[1], dz = ez * p->ng.h[2];
        cd g = g0(std::sqrt(dx * dx + dy * dy + dz * dz), p->lat.k0);
        g0t[k] = cmake<double>(g.real(), g.imag());
      }
  cplx<double>* dg0 = nullptr;
  CHK(upload(p, &dg0, g0t));
  if (p->sym) CHK(build_sym(p, start, pos3_dev, dg0, ca, st));
  // count, scan, fill one CSR: rows are one point set (stencils s3r,
  // weights u3r, positions posr, box sort rstart), columns the other
  const bool cv = p->complex_kernel;
  const size_t vb = cv ? 16 : 8;
  struct Csr {
    int64_t* rowptr = nullptr;
    int32_t* col = nullptr;
    void* val = nullptr;
    void* val_adj = nullptr;
    int32_t* order = nullptr;
    int64_t slots = 0, nnz = 0;
    std::vector<int64_t> host_rowptr;
  };
  auto build_csr = [&](CorrArgs a, int64_t nr, const int32_t* s3r, const double* u3r, const double* posr,
                       const std::vector<int32_t>& rstart, int64_t nc, const double* u3c, const double* posc,
                       const int32_t* cstart, bool with_adj, Csr& out) -> int {
    a.N = nr;
    a.Nc = nc;
    int64_t* dcount = nullptr;
    CHK(dalloc(p, &dcount, nr));
    CHK(launch_corr_count(a, s3r, cstart, dcount, st));
    std::vector<int64_t>& rowptr = out.host_rowptr;
    rowptr.assign(nr + 1, 0);
    HIPCHK(hipMemcpyAsync(rowptr.data() + 1, dcount, nr * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int64_t m = 0; m < nr; ++m) rowptr[m + 1] += rowptr[m];
    out.nnz = rowptr[nr];
    if (std::getenv("FFTPIM_LOG"))
      std::fprintf(stderr, "fftpim plan: correction nnz %lld\n", static_cast<long long>(out.nnz));
    CHK(upload(p, &out.rowptr, rowptr));
    {
      std::vector<int32_t> order;
      build_row_order(rstart, p->nb, nr, order);
      out.slots = static_cast<int64_t>(order.size());
      CHK(upload(p, &out.order, order));
    }
    CHK(dalloc(p, &out.col, out.nnz));
    unsigned char* v = nullptr;
    CHK(dalloc(p, &v, out.nnz * vb));
    out.val = v;
    if (with_adj) {
      unsigned char* va = nullptr;
      CHK(dalloc(p, &va, out.nnz * vb));
      out.val_adj = va;
    }
    CHK(launch_corr_fill(q, cv, with_adj, a, s3r, u3r, posr, u3c, posc, cstart, dg0, out.rowptr, out.col, out.val,
                         out.val_adj, st));
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipGetLastError());
    dfree(p, dcount);
    return FFTPIM_OK;
  };
  Csr fwd;
  if (!p->sep) {
    CHK(build_csr(ca, p->N, p->near_s, p->near_u, pos3_dev, start, p->N, p->near_u, pos3_dev, p->box_start,
                  p->nonhermitian, fwd));
  } else {
    // rows are observers; the conjugate transpose gets its own CSR with
    // source rows: C^H(n, m) = conj(C(m, n)) is the conjugate-transpose
    // value of the fill with the roles swapped (the region and G0 are
    // symmetric under swapping the points and reversing the image), and for
    // a real symmetric kernel simply the swapped fill's value
    CHK(build_csr(ca, p->No, p->near_s_o, p->near_u_o, pos3_o, *start_o, p->N, p->near_u, pos3_dev, p->box_start,
                  false, fwd));
    Csr adj;
    CHK(build_csr(ca, p->N, p->near_s, p->near_u, pos3_dev, start, p->No, p->near_u_o, pos3_o, p->box_start_o,
                  p->nonhermitian, adj));
    p->rowptr_a = adj.rowptr;
    p->col_a = adj.col;
    if (p->nonhermitian) {
      p->val_a = adj.val_adj;
      dfree(p, adj.val);
    } else {
      p->val_a = adj.val;
    }
    p->corr_order_a = adj.order;
    p->corr_slots_a = adj.slots;
    p->nnz_a = adj.nnz;
  }
  p->rowptr = fwd.rowptr;
  p->col = fwd.col;
  p->val = fwd.val;
  p->val_adj = fwd.val_adj;
  p->corr_order = fwd.order;
  p->corr_slots = fwd.slots;
  p->nnz = fwd.nnz;
  const std::vector<int64_t>& rowptr = fwd.host_rowptr;
  // the traversal arrays (per-axis candidate lists, image phases, G0 table)
  // stay with the plan: the position gradient walks the same pairs
  p->grad_ca = ca;
  p->grad_ca.images_only = 0;
  p->g0tab = dg0;
  if (p->tile) CHK(build_tiles(p, start, rowptr, st));
  return FFTPIM_OK;
}

void plan_log(const char* what, std::chrono::steady_clock::time_point t0) {
  static const bool on = std::getenv("FFTPIM_LOG") != nullptr;
  if (!on) return;
  double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  std::fprintf(stderr, "fftpim plan: %-28s %8.3f s\n", what, s);
  std::fflush(stderr);
}

int build_plan(fftpim_plan_s* p, int64_t N, const double* src_dev, int64_t No, const double* obs_dev,
               hipStream_t st) {
  const auto t0 = std::chrono::steady_clock::now();
  const fftpim_problem_t& pr = p->problem;
  const fftpim_params_t& pm = p->prm;
  const int dims = pr.periodic_dims;
  const bool sep = obs_dev != nullptr;
  p->sep = sep;
  p->No = sep ? No : N;
  // positions to host
  std::vector<double> xyz(static_cast<size_t>(N) * 3), xyz_o;
  HIPCHK(hipMemcpyAsync(xyz.data(), src_dev, xyz.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  if (sep) {
    xyz_o.resize(static_cast<size_t>(No) * 3);
    HIPCHK(hipMemcpyAsync(xyz_o.data(), obs_dev, xyz_o.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  // target region D (Sec. 3.2): the cell on periodic axes; the given box or
  // the bounding box of sources and observers elsewhere
  double lo[3], hi[3];
  for (int c = 0; c < 3; ++c) {
    double mn = INFINITY, mx = -INFINITY;
    for (const std::vector<double>* X : {&xyz, &xyz_o})
      for (size_t i = 0; i < X->size() / 3; ++i) {
        const double v = (*X)[3 * i + c];
        if (!std::isfinite(v)) return FFTPIM_ERR_INVALID_ARG;
        mn = std::min(mn, v);
        mx = std::max(mx, v);
      }
    if (c < dims) {
      if (mn < 0.0 || mx >= pr.L[c]) return FFTPIM_ERR_OUT_OF_CELL;
      lo[c] = 0.0;
      hi[c] = pr.L[c];
    } else if (pr.has_box) {
      if (mn < pr.box_lo[c] || mx > pr.box_hi[c] || !(pr.box_hi[c] > pr.box_lo[c])) return FFTPIM_ERR_OUT_OF_CELL;
      lo[c] = pr.box_lo[c];
      hi[c] = pr.box_hi[c];
    } else {
      lo[c] = mn;
      hi[c] = mx > mn ? mx : mn + 1.0;
    }
  }
  // near grid (Sec. 3.3): n - q cells on periodic axes, n - q - 1 otherwise
  GridGeom& g = p->ng;
  g.q = pm.near_order;
  for (int c = 0; c < 3; ++c) {
    g.n[c] = pm.near_n[c];
    g.nint[c] = c < dims ? g.n[c] - g.q : g.n[c] - g.q - 1;
    if (g.nint[c] < 1) return FFTPIM_ERR_INVALID_ARG;
    g.h[c] = (hi[c] - lo[c]) / g.nint[c];
    g.origin[c] = lo[c] - 0.5 * (g.q - 1) * g.h[c];
    g.lo[c] = lo[c];
    // the zero-padded (aperiodic) convolution needs M >= 2 n - 1 points
    p->M[c] = fft_length(2 * g.n[c] - 1);
    p->nb[c] = g.nint[c] + 1;
  }
  if (pm.corr_ball > 0.0) {
    // every pair of boxes with overlapping stencils (offsets up to q on each
    // axis) must be corrected: the near table's zeroed entries reach them
    const CorrRegion reg = corr_region(p);
    if (!ball_close(reg.bw, reg.br2, g.q, g.q, g.q)) return FFTPIM_ERR_INVALID_ARG;
    for (int c = 0; c < 3; ++c)
      if (reg.reach[c] > kMaxCorrRadius) return FFTPIM_ERR_INVALID_ARG;
  }
  // far grids (Sec. 3.2, Eq. (grid)): n - q - 1 cells on every axis
  GridGeom& f = p->fg;
  f.q = pm.far_order;
  for (int c = 0; c < 3; ++c) {
    f.n[c] = pm.far_n[c];
    f.nint[c] = f.n[c] - f.q - 1;
    if (f.nint[c] < 1) return FFTPIM_ERR_INVALID_ARG;
    f.h[c] = (hi[c] - lo[c]) / f.nint[c];
    f.origin[c] = lo[c] - 0.5 * (f.q - 1) * f.h[c];
    f.lo[c] = lo[c];
    p->fnb[c] = f.nint[c] + 1;
  }
  // far grid sum: direct (term by term or matrix cores) or FFT convolution
  {
    const int64_t ngf = static_cast<int64_t>(f.n[0]) * f.n[1] * f.n[2];
    const bool bf16 = pm.precision == FFTPIM_F32_FARBF16 || pm.precision == FFTPIM_F32_FARBF16X3;
    p->far_fft = pm.far_sum == FFTPIM_FAR_FFT || (pm.far_sum == FFTPIM_FAR_AUTO && !bf16 && ngf >= kFarFftMinNodes);
    for (int c = 0; c < 3; ++c) p->Mf[c] = p->far_fft ? fft_length(2 * f.n[c] - 1) : 0;
  }
  // near stencils and the box sort of one point set (Sec. 3.3), with its
  // stencils on one far grid (Sec. 3.2, Eq. (grid)): the source grid, or the
  // observer grid shifted by -h/2
  struct SetGeom {
    int64_t n = 0;
    std::vector<int32_t> order, start, s_sorted, f_s, forder, fstart;
    std::vector<double> u_sorted, pos_sorted, f_u;
    int fmax = 0;
  };
  const int64_t nboxes = static_cast<int64_t>(p->nb[0]) * p->nb[1] * p->nb[2];
  const int64_t fboxes = static_cast<int64_t>(p->fnb[0]) * p->fnb[1] * p->fnb[2];
  auto near_geom = [&](const std::vector<double>& X, SetGeom& G) {
    const int64_t n = static_cast<int64_t>(X.size() / 3);
    G.n = n;
    std::vector<int32_t> sv(3 * n);
    std::vector<double> uv(3 * n);
    std::vector<int64_t> key(n);
    for (int64_t i = 0; i < n; ++i) {
      for (int c = 0; c < 3; ++c) stencil(X[3 * i + c], g.origin[c], g.h[c], g.q, g.n[c], sv[3 * i + c], uv[3 * i + c]);
      key[i] = (static_cast<int64_t>(sv[3 * i]) * p->nb[1] + sv[3 * i + 1]) * p->nb[2] + sv[3 * i + 2];
    }
    counting_sort(key, nboxes, G.order, G.start);
    G.s_sorted.resize(3 * n);
    G.u_sorted.resize(3 * n);
    G.pos_sorted.resize(3 * n);
    for (int64_t j = 0; j < n; ++j) {
      const int64_t i = G.order[j];
      for (int c = 0; c < 3; ++c) {
        G.s_sorted[c * n + j] = sv[3 * i + c];
        G.u_sorted[c * n + j] = uv[3 * i + c];
        G.pos_sorted[c * n + j] = X[3 * i + c];
      }
    }
  };
  auto far_geom = [&](SetGeom& G, double shift, std::vector<int32_t>& fs, std::vector<double>& fu,
                      std::vector<int32_t>& forder, std::vector<int32_t>& fstart, int& fmax) {
    const int64_t n = G.n;
    fs.resize(3 * n);
    fu.resize(3 * n);
    std::vector<int64_t> fkey(n);
    for (int64_t j = 0; j < n; ++j) {
      for (int c = 0; c < 3; ++c)
        stencil(G.pos_sorted[c * n + j], f.origin[c] + shift * f.h[c], f.h[c], f.q, f.n[c], fs[c * n + j], fu[c * n + j]);
      fkey[j] = (static_cast<int64_t>(fs[j]) * p->fnb[1] + fs[n + j]) * p->fnb[2] + fs[2 * n + j];
    }
    counting_sort(fkey, fboxes, forder, fstart);
    fmax = 0;
    for (int64_t k = 0; k < fboxes; ++k) fmax = std::max(fmax, fstart[k + 1] - fstart[k]);
  };
  SetGeom gs, go;
  near_geom(xyz, gs);
  if (sep) near_geom(xyz_o, go);
  SetGeom& gobs = sep ? go : gs;
  std::vector<int32_t> fs_s, fo_s, forder_s, fstart_s, forder_o, fstart_o;
  std::vector<double> fs_u, fo_u;
  far_geom(gs, 0.0, fs_s, fs_u, forder_s, fstart_s, p->fmax_box_s);
  far_geom(gobs, -0.5, fo_s, fo_u, forder_o, fstart_o, p->fmax_box_o);
  const std::vector<int32_t>& order = gs.order;
  const std::vector<int32_t>& start = gs.start;
  const std::vector<int32_t>& s_sorted = gs.s_sorted;
  const std::vector<double>& u_sorted = gs.u_sorted;
  const std::vector<double>& pos_sorted = gs.pos_sorted;

  CHK(upload(p, &p->perm, order));
  CHK(upload(p, &p->near_s, s_sorted));
  CHK(upload(p, &p->near_u, u_sorted));
  CHK(upload(p, &p->box_start, start));
  CHK(upload(p, &p->fs_s, fs_s));
  CHK(upload(p, &p->fs_u, fs_u));
  CHK(upload(p, &p->fo_s, fo_s));
  CHK(upload(p, &p->fo_u, fo_u));
  const std::vector<double> w_near = weights_soa(u_sorted, N, g.q);
  CHK(upload(p, &p->near_w, w_near));
  double* dpos_o = nullptr;
  if (sep) {
    CHK(upload(p, &p->perm_o, go.order));
    CHK(upload(p, &p->near_s_o, go.s_sorted));
    CHK(upload(p, &p->near_u_o, go.u_sorted));
    CHK(upload(p, &p->box_start_o, go.start));
    CHK(upload(p, &p->near_w_o, weights_soa(go.u_sorted, No, g.q)));
    CHK(upload(p, &dpos_o, go.pos_sorted));
  } else {
    p->perm_o = p->perm;
    p->near_s_o = p->near_s;
    p->near_u_o = p->near_u;
    p->near_w_o = p->near_w;
    p->box_start_o = p->box_start;
  }
  // the node-major projection weights serve sources only: with separate
  // observers the conjugate transpose projects observers, so both use the
  // box-tiled gather
  if (!sep && planes_for(p, pm.nrhs_max) <= kSpreadCsrPlanes) {
    // W^T by grid node (Step 1 of Sec. 3.3 as a sparse product): entries of a
    // node in increasing point order, weight = product of the 1D weights
    const int K1 = g.q + 1;
    const int64_t n3 = static_cast<int64_t>(g.n[0]) * g.n[1] * g.n[2];
    std::vector<int64_t> wrow(n3 + 1, 0);
    auto node_of = [&](int64_t m, int a, int b, int c) {
      return (static_cast<int64_t>(s_sorted[m] + a) * g.n[1] + (s_sorted[N + m] + b)) * g.n[2] + (s_sorted[2 * N + m] + c);
    };
    for (int64_t m = 0; m < N; ++m)
      for (int a = 0; a < K1; ++a)
        for (int b = 0; b < K1; ++b)
          for (int c = 0; c < K1; ++c) wrow[node_of(m, a, b, c) + 1]++;
    for (int64_t k = 0; k < n3; ++k) wrow[k + 1] += wrow[k];
    std::vector<int64_t> cur(wrow.begin(), wrow.end() - 1);
    std::vector<int32_t> widx(static_cast<size_t>(wrow[n3]));
    std::vector<double> wval(static_cast<size_t>(wrow[n3]));
    for (int64_t m = 0; m < N; ++m)
      for (int a = 0; a < K1; ++a)
        for (int b = 0; b < K1; ++b)
          for (int c = 0; c < K1; ++c) {
            const int64_t k = cur[node_of(m, a, b, c)]++;
            widx[k] = static_cast<int32_t>(m);
            wval[k] = w_near[a * N + m] * w_near[(K1 + b) * N + m] * w_near[(2 * K1 + c) * N + m];
          }
    // clustered points leave most of a fine grid empty: then only the nodes
    // with entries are listed and visited (the grid is zeroed first);
    // otherwise every node is visited and writes its own value
    int64_t filled = 0;
    for (int64_t k = 0; k < n3; ++k) filled += wrow[k + 1] > wrow[k] ? 1 : 0;
    if (filled > 0 && 2 * filled < n3) {
      std::vector<int64_t> wnode, wrow_c;
      wnode.reserve(static_cast<size_t>(filled));
      wrow_c.reserve(static_cast<size_t>(filled) + 1);
      for (int64_t k = 0; k < n3; ++k)
        if (wrow[k + 1] > wrow[k]) {
          wnode.push_back(k);
          wrow_c.push_back(wrow[k]);
        }
      wrow_c.push_back(wrow[n3]);
      p->wt_nnodes = filled;
      CHK(upload(p, &p->wt_node, wnode));
      CHK(upload(p, &p->wt_row, wrow_c));
    } else {
      p->wt_nnodes = n3;
      CHK(upload(p, &p->wt_row, wrow));
    }
    CHK(upload(p, &p->wt_idx, widx));
    CHK(upload(p, &p->wt_val, wval));
  }
  CHK(upload(p, &p->fs_w, weights_soa(fs_u, N, f.q)));
  CHK(upload(p, &p->fo_w, weights_soa(fo_u, p->No, f.q)));
  CHK(upload(p, &p->fperm_s, forder_s));
  CHK(upload(p, &p->fbox_start_s, fstart_s));
  CHK(upload(p, &p->fperm_o, forder_o));
  CHK(upload(p, &p->fbox_start_o, fstart_o));
  double* dpos = nullptr;
  CHK(upload(p, &dpos, pos_sorted));

  plan_log("geometry and sort", t0);
  if (pm.precision != FFTPIM_F64)
    CHK(build_tables<float>(p, st));
  else
    CHK(build_tables<double>(p, st));
  plan_log("near and far tables", t0);
  // correction layout: symmetric box-pair blocks when boxes hold several
  // points each and a box's amplitudes fit the kernel's LDS staging
  {
    int64_t nonempty = 0;
    int max_box = 0;
    for (int64_t b = 0; b < nboxes; ++b) {
      const int cnt = start[b + 1] - start[b];
      nonempty += cnt > 0;
      max_box = std::max(max_box, cnt);
    }
    const int Pm = planes_for(p, pm.nrhs_max);
    // LDS: the fill stages a (2q+1)^3 complex table slice, the apply stages a
    // box's amplitudes and row sums
    const bool fits = static_cast<int64_t>(max_box) * Pm <= 2048 && g.q <= 7;
    const bool dense = static_cast<double>(N) >= 3.0 * static_cast<double>(std::max<int64_t>(nonempty, 1));
    if (sep) {
      // the box-pair blocks and the dense tiles rely on the correction being
      // symmetric in observer and source: separate observers use the CSR
      if (pm.corr_layout != FFTPIM_CORR_AUTO && pm.corr_layout != FFTPIM_CORR_CSR) return FFTPIM_ERR_UNSUPPORTED;
    } else if (pm.corr_layout == FFTPIM_CORR_SYM) {
      if (!fits) return FFTPIM_ERR_INVALID_ARG;
      p->sym = true;
    } else if (pm.corr_layout == FFTPIM_CORR_TILE) {
      if (p->complex_kernel) return FFTPIM_ERR_UNSUPPORTED;
      p->tile = true;
    } else if (pm.corr_layout == FFTPIM_CORR_AUTO) {
      // many planes re-read a value per plane in the box-pair kernel; the
      // dense tiles take them on the matrix cores (real values only)
      p->tile = !p->complex_kernel && Pm >= 8;
      p->sym = !p->tile && fits && dense && Pm <= 4;
    }
  }
  CHK(build_correction(p, start, dpos, sep ? &go.start : nullptr, dpos_o, st));
  plan_log("correction operator", t0);
  p->pos3 = dpos;  // kept for the exact terms of the position gradient
  if (dpos_o) dfree(p, dpos_o);

  // workspace
  const int P = planes_for(p, pm.nrhs_max);
  p->nplanes_max = P;
  const size_t es = cbytes(p);
  // packed inputs and the three parts hold either point set
  const size_t Nmax = static_cast<size_t>(std::max(N, p->No));
  unsigned char* b = nullptr;
  CHK(dalloc(p, &b, Nmax * P * es));
  p->q_int = b;
  CHK(dalloc(p, &b, Nmax * P * es));
  p->u_int = b;
  CHK(dalloc(p, &b, Nmax * P * es));
  p->u_corr = b;
  CHK(dalloc(p, &b, Nmax * P * es));
  p->u_far = b;
  HIPCHK(hipStreamCreateWithFlags(&p->s_corr, hipStreamNonBlocking));
  HIPCHK(hipStreamCreateWithFlags(&p->s_far, hipStreamNonBlocking));
  HIPCHK(hipStreamCreateWithFlags(&p->s_near, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&p->ev_corr, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&p->ev_far, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&p->ev_near, hipEventDisableTiming));
  CHK(alloc_work_set(p, p->ws));
  if (p->sym) {
    // partial sums for twice the planes: the fused forward + adjoint pair
    // carries both inputs through one pass
    CHK(dalloc(p, &b, static_cast<size_t>(std::max<int64_t>(p->symd.yslots, 1)) * 2 * P * 16));
    p->sym_ypart = b;
    CHK(dalloc(p, &b, static_cast<size_t>(std::max<int64_t>(p->symd.zslots, 1)) * 2 * P * 16));
    p->sym_zpart = b;
  }
  CHK(dalloc(p, &p->sums, static_cast<size_t>(6) * P));
  CHK(dalloc(p, &p->sums_work, static_cast<size_t>(plane_sums_chunks(static_cast<int64_t>(Nmax))) * P * 4));
  CHK(dalloc(p, &p->status_dev, 1));
  HIPCHK(hipMemsetAsync(p->status_dev, 0, sizeof(int), st));
  HIPCHK(hipStreamSynchronize(st));
  return FFTPIM_OK;
}

Lattice lattice_of(const fftpim_problem_t& pr) {
  Lattice lat{};
  lat.dims = pr.periodic_dims;
  for (int c = 0; c < 3; ++c) {
    lat.L[c] = c < lat.dims ? pr.L[c] : 1.0;
    lat.kt[c] = c < lat.dims ? cd(pr.kt[c], pr.kt_im[c]) : cd(0.0, 0.0);
  }
  lat.k0 = cd(pr.k0, pr.k0_im);
  return lat;
}

// ---------------------------------------------------------------------------
// Allocation-free fused pair: the pair's own arrays (a second work set, the
// packed adjoint input, the three parts of A^H v) are laid out in a fixed
// per-device array instead of plan-owned allocations.
// ---------------------------------------------------------------------------

constexpr size_t kScratchBytes = size_t{64} << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the given device, looked up once per device
// with that device current (each device holds its own copy of the array; in
// host code the array's name is not a device address).
int scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return FFTPIM_ERR_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device] == nullptr) {
    int cur = -1;
    HIPCHK(hipGetDevice(&cur));
    if (cur != device) HIPCHK(hipSetDevice(device));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || ptr == nullptr) return FFTPIM_ERR_DEVICE;
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return FFTPIM_OK;
}

// No C++ exception may cross the C ABI: host allocations (std::vector) and
// the far-table worker threads can throw on resource exhaustion.
template <typename F>
int guarded(F&& f) noexcept {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return FFTPIM_ERR_NO_MEMORY;
  } catch (const std::length_error&) {
    return FFTPIM_ERR_NO_MEMORY;
  } catch (const std::system_error&) {
    return FFTPIM_ERR_NO_MEMORY;  // e.g. no host thread could be started
  } catch (...) {
    return FFTPIM_ERR_DEVICE;
  }
}

}  // namespace

extern "C" {

int fftpim_default_params(const fftpim_problem_t* problem, fftpim_params_t* params) {
  return guarded([&]() -> int {
    if (!problem || !params) return FFTPIM_ERR_INVALID_ARG;
    fftpim_params_t p{};
    for (int c = 0; c < 3; ++c) {
      p.near_n[c] = 16;
      p.far_n[c] = 16;
    }
    p.near_order = 4;
    p.corr_radius = 6;
    p.far_order = 7;
    p.n_images = 1;
    p.precision = FFTPIM_F64;
    p.value_type = FFTPIM_COMPLEX;
    p.self_mode = FFTPIM_SELF_IMAGES;
    p.order_io = FFTPIM_ORDER_USER;
    p.nrhs_max = 1;
    p.corr_layout = FFTPIM_CORR_AUTO;
    *params = p;
    return FFTPIM_OK;
  });
}

int fftpim_plan(fftpim_plan_t* plan, const fftpim_problem_t* problem, const fftpim_params_t* params,
                int64_t n_src, const double* src_xyz_dev, int64_t n_obs, const double* obs_xyz_dev,
                fftpim_stream_t stream) {
  return guarded([&]() -> int {
    if (!plan || !problem || !params || !src_xyz_dev) return FFTPIM_ERR_INVALID_ARG;
    *plan = nullptr;
    if (n_src < 1 || n_src > (int64_t{1} << 30)) return FFTPIM_ERR_INVALID_ARG;
    if (obs_xyz_dev != nullptr) {
      // separate observers: the self term of Eq. (5) has no meaning
      if (n_obs < 1 || n_obs > (int64_t{1} << 30)) return FFTPIM_ERR_INVALID_ARG;
      if (params->self_mode != FFTPIM_SELF_IMAGES) return FFTPIM_ERR_INVALID_ARG;
    } else if (n_obs != n_src && n_obs != 0) {
      return FFTPIM_ERR_INVALID_ARG;
    }
    CHK(validate(problem, params));
    const Lattice lat = lattice_of(*problem);
    if (params->value_type == FFTPIM_REAL && !lat.npsp()) return FFTPIM_ERR_INVALID_ARG;
    if (check_supported(lat)) return FFTPIM_ERR_UNSUPPORTED;
    if (wood_anomaly(lat)) return FFTPIM_ERR_WOOD_ANOMALY;
    auto t0 = std::chrono::steady_clock::now();
    fftpim_plan_s* p = new (std::nothrow) fftpim_plan_s();
    if (!p) return FFTPIM_ERR_NO_MEMORY;
    p->lat = lat;
    p->problem = *problem;
    p->prm = *params;
    p->N = n_src;
    HIPCHK(hipGetDevice(&p->device));
    p->complex_kernel = !lat.npsp();
    p->nonhermitian = !lat.hermitian();
    if (params->self_mode == FFTPIM_SELF_EXCLUDE) p->self_coef = pgf_self(lat);
    hipStream_t st = static_cast<hipStream_t>(stream);
    // an exception inside the build still frees the partly built plan
    int s = guarded([&]() -> int { return build_plan(p, n_src, src_xyz_dev, n_obs, obs_xyz_dev, st); });
    if (s != FFTPIM_OK) {
      fftpim_destroy(p);
      return s;
    }
    p->plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    p->last_stream = st;
    if (std::getenv("FFTPIM_LOG")) {
      std::fprintf(stderr, "fftpim plan: N=%lld near %dx%dx%d q=%d rc=%d far %dx%dx%d q=%d nnz=%lld bytes=%lld %.3fs\n",
                   static_cast<long long>(p->N), p->ng.n[0], p->ng.n[1], p->ng.n[2], p->ng.q, p->prm.corr_radius,
                   p->fg.n[0], p->fg.n[1], p->fg.n[2], p->fg.q, static_cast<long long>(p->nnz),
                   static_cast<long long>(p->device_bytes), p->plan_seconds);
    }
    *plan = p;
    return FFTPIM_OK;
  });
}

int fftpim_apply(fftpim_plan_t plan, const void* q_dev, void* u_dev, int nrhs, fftpim_stream_t stream) {
  return guarded([&]() -> int {
    return apply_common(plan, FFTPIM_PART_ALL, 0, q_dev, u_dev, nrhs, stream, true);
  });
}

int fftpim_apply_adjoint(fftpim_plan_t plan, const void* v_dev, void* w_dev, int nrhs, fftpim_stream_t stream) {
  return guarded([&]() -> int {
    return apply_common(plan, FFTPIM_PART_ALL, 1, v_dev, w_dev, nrhs, stream, true);
  });
}

int fftpim_apply_pair(fftpim_plan_t plan, const void* q_dev, void* u_dev, const void* v_dev, void* w_dev, int nrhs,
                      fftpim_stream_t stream) {
  return guarded([&]() -> int {
    if (!plan || !q_dev || !u_dev || !v_dev || !w_dev) return FFTPIM_ERR_INVALID_ARG;
    if (nrhs < 1 || nrhs > plan->prm.nrhs_max) return FFTPIM_ERR_INVALID_ARG;
    if (plan->sep) return FFTPIM_ERR_UNSUPPORTED;
    hipStream_t st = static_cast<hipStream_t>(stream);
    CHK(ensure_pair_buffers(plan));
    if (plan->prm.precision != FFTPIM_F64)
      return run_apply_pair<float>(plan, plan->pair, q_dev, u_dev, v_dev, w_dev, nrhs, st);
    return run_apply_pair<double>(plan, plan->pair, q_dev, u_dev, v_dev, w_dev, nrhs, st);
  });
}

int fftpim_apply_pair_noalloc(fftpim_plan_t plan, const void* q_dev, void* u_dev, const void* v_dev, void* w_dev,
                              int nrhs, fftpim_stream_t stream) {
  return guarded([&]() -> int {
    if (!plan || !q_dev || !u_dev || !v_dev || !w_dev) return FFTPIM_ERR_INVALID_ARG;
    if (nrhs < 1 || nrhs > plan->prm.nrhs_max) return FFTPIM_ERR_INVALID_ARG;
    if (plan->sep) return FFTPIM_ERR_UNSUPPORTED;
    if (pair_buffer_bytes(plan) > kScratchBytes) return FFTPIM_ERR_SCRATCH_LIMIT;
    void* base = nullptr;
    CHK(scratch_address(plan->device, &base));
    const PairBufs pb = carve_pair_buffers(plan, static_cast<unsigned char*>(base));
    hipStream_t st = static_cast<hipStream_t>(stream);
    // stage timing may grow its event pool: it is off for this call
    const bool timing = plan->timing;
    plan->timing = false;
    const int s = plan->prm.precision != FFTPIM_F64
                      ? run_apply_pair<float>(plan, pb, q_dev, u_dev, v_dev, w_dev, nrhs, st)
                      : run_apply_pair<double>(plan, pb, q_dev, u_dev, v_dev, w_dev, nrhs, st);
    plan->timing = timing;
    return s;
  });
}

int fftpim_grad_positions(fftpim_plan_t plan, const void* q_dev, const void* g_dev, int nrhs, double* grad_dev,
                          fftpim_stream_t stream) {
  return guarded([&]() -> int {
    if (!plan || !q_dev || !g_dev || !grad_dev) return FFTPIM_ERR_INVALID_ARG;
    if (nrhs < 1 || nrhs > plan->prm.nrhs_max) return FFTPIM_ERR_INVALID_ARG;
    if (plan->g0tab == nullptr || plan->pos3 == nullptr || plan->sep) return FFTPIM_ERR_UNSUPPORTED;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (plan->prm.precision != FFTPIM_F64) return run_grad<float>(plan, q_dev, g_dev, nrhs, grad_dev, st);
    return run_grad<double>(plan, q_dev, g_dev, nrhs, grad_dev, st);
  });
}

int fftpim_apply_parts(fftpim_plan_t plan, int parts, int adjoint, const void* q_dev, void* u_dev, int nrhs,
                       fftpim_stream_t stream) {
  return guarded([&]() -> int {
    return apply_common(plan, parts, adjoint, q_dev, u_dev, nrhs, stream, false);
  });
}

int fftpim_get_permutation(fftpim_plan_t plan, int which, int32_t* perm_dev) {
  return guarded([&]() -> int {
    if (!plan || !perm_dev || (which != 0 && which != 1)) return FFTPIM_ERR_INVALID_ARG;
    if (which == 1)
      HIPCHK(hipMemcpy(perm_dev, plan->perm_o, plan->No * sizeof(int32_t), hipMemcpyDeviceToDevice));
    else
      HIPCHK(hipMemcpy(perm_dev, plan->perm, plan->N * sizeof(int32_t), hipMemcpyDeviceToDevice));
    return FFTPIM_OK;
  });
}

int fftpim_plan_info(fftpim_plan_t plan, fftpim_info_t* info) {
  return guarded([&]() -> int {
    if (!plan || !info) return FFTPIM_ERR_INVALID_ARG;
    fftpim_info_t r{};
    r.n_src = plan->N;
    r.n_obs = plan->No;
    for (int c = 0; c < 3; ++c) {
      r.near_n[c] = plan->ng.n[c];
      r.near_fft[c] = plan->M[c];
      r.near_cells[c] = plan->ng.nint[c];
      r.near_h[c] = plan->ng.h[c];
      r.domain_lo[c] = plan->ng.lo[c];
      r.domain_hi[c] = plan->ng.lo[c] + plan->ng.h[c] * plan->ng.nint[c];
      r.far_n[c] = plan->fg.n[c];
      r.far_cells[c] = plan->fg.nint[c];
      r.far_h[c] = plan->fg.h[c];
      r.far_fft[c] = plan->Mf[c];
    }
    r.corr_nnz = plan->nnz + plan->nnz_a + plan->sym_nvals;
    r.corr_sym_values = plan->sym_nvals;
    r.corr_csr_nnz = plan->tile ? 0 : plan->nnz + plan->nnz_a;
    r.corr_tile_values = plan->tile_nvals;
    r.corr_value_bytes = plan->complex_kernel ? 16 : 8;
    r.corr_layout_used = plan->tile ? FFTPIM_CORR_TILE : (plan->sym ? FFTPIM_CORR_SYM : FFTPIM_CORR_CSR);
    r.device_bytes = plan->device_bytes;
    r.nplanes_max = plan->nplanes_max;
    r.plan_seconds = plan->plan_seconds;
    *info = r;
    return FFTPIM_OK;
  });
}

int fftpim_last_status(fftpim_plan_t plan) {
  return guarded([&]() -> int {
    if (!plan) return FFTPIM_ERR_INVALID_ARG;
    HIPCHK(hipStreamSynchronize(plan->last_stream));
    int v = 0;
    HIPCHK(hipMemcpy(&v, plan->status_dev, sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemset(plan->status_dev, 0, sizeof(int)));
    return v;
  });
}

int fftpim_stage_times(fftpim_plan_t plan, int enable, double* ms_out, int64_t* calls_out) {
  return guarded([&]() -> int {
    if (!plan) return FFTPIM_ERR_INVALID_ARG;
    resolve_timers(plan);
    if (ms_out)
      for (int s = 0; s < FFTPIM_NSTAGES; ++s) ms_out[s] = plan->stage_ms[s];
    if (calls_out)
      for (int s = 0; s < FFTPIM_NSTAGES; ++s) calls_out[s] = plan->stage_calls[s];
    if (enable) {
      for (int s = 0; s < FFTPIM_NSTAGES; ++s) {
        plan->stage_ms[s] = 0.0;
        plan->stage_calls[s] = 0;
      }
    }
    plan->timing = enable != 0;
    return FFTPIM_OK;
  });
}

int fftpim_destroy(fftpim_plan_t plan) {
  return guarded([&]() -> int {
    if (!plan) return FFTPIM_OK;
    // the plan's streams may still be reading its buffers (teardown goes on
    // whatever these calls return)
    for (hipStream_t s : {plan->s_corr, plan->s_far, plan->s_near})
      if (s) (void)hipStreamSynchronize(s);
    (void)hipStreamSynchronize(plan->last_stream);
    for (hipEvent_t e : plan->ev_pool) (void)hipEventDestroy(e);
    plan->ev_pool.clear();
    for (hipEvent_t e : {plan->ev_fork, plan->ev_corr, plan->ev_far, plan->ev_near})
      if (e) (void)hipEventDestroy(e);
    for (hipStream_t s : {plan->s_corr, plan->s_far, plan->s_near})
      if (s) (void)hipStreamDestroy(s);
    for (const DevBuf& b : plan->allocations) (void)hipFree(b.p);
    plan->allocations.clear();
    delete plan;
    return FFTPIM_OK;
  });
}

const char* fftpim_error_string(int status) {
  switch (status) {
    case FFTPIM_OK: return "success";
    case FFTPIM_ERR_INVALID_ARG: return "invalid argument";
    case FFTPIM_ERR_OUT_OF_CELL: return "a point lies outside the zeroth cell or the given box";
    case FFTPIM_ERR_NOT_NEUTRAL: return "static no-phase problem with a non-neutral right-hand side";
    case FFTPIM_ERR_WOOD_ANOMALY: return "a Floquet wavenumber vanishes (Rayleigh-Wood anomaly)";
    case FFTPIM_ERR_UNSUPPORTED: return "problem class not supported by this library";
    case FFTPIM_ERR_NO_MEMORY: return "out of memory";
    case FFTPIM_ERR_DEVICE: return "HIP runtime error";
    case FFTPIM_ERR_UNIMPLEMENTED: return "not implemented";
    case FFTPIM_ERR_SCRATCH_LIMIT:
      return "the plan's pair work arrays exceed the 64 MiB per-device array of fftpim_apply_pair_noalloc";
    default: return "unknown status";
  }
}

int fftpim_eval_pgf(const fftpim_problem_t* problem, int64_t n, const double* r_xyz, double* out) {
  return guarded([&]() -> int {
    if (!problem || !r_xyz || !out || n < 0) return FFTPIM_ERR_INVALID_ARG;
    if (problem->periodic_dims < 1 || problem->periodic_dims > 3) return FFTPIM_ERR_INVALID_ARG;
    const Lattice lat = lattice_of(*problem);
    if (check_supported(lat)) return FFTPIM_ERR_UNSUPPORTED;
    for (int64_t i = 0; i < n; ++i) {
      cd v = pgf(lat, r_xyz + 3 * i);
      out[2 * i] = v.real();
      out[2 * i + 1] = v.imag();
    }
    return FFTPIM_OK;
  });
}

int fftpim_eval_pgf_self(const fftpim_problem_t* problem, double* out) {
  return guarded([&]() -> int {
    if (!problem || !out) return FFTPIM_ERR_INVALID_ARG;
    if (problem->periodic_dims < 1 || problem->periodic_dims > 3) return FFTPIM_ERR_INVALID_ARG;
    const Lattice lat = lattice_of(*problem);
    if (check_supported(lat)) return FFTPIM_ERR_UNSUPPORTED;
    if (wood_anomaly(lat)) return FFTPIM_ERR_WOOD_ANOMALY;
    const cd v = pgf_self(lat);
    out[0] = v.real();
    out[1] = v.imag();
    return FFTPIM_OK;
  });
}

}  // extern "C"
