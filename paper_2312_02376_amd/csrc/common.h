// Shared definitions of the FFT-PIM library: complex helpers, grid geometry and
// the plan object.  Device code targets gfx950 (CDNA4, 64-wide wavefronts).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fftpim.h"
#include "pgf_host.h"

namespace fftpim {

template <typename R>
struct cplx {
  R x, y;
};

template <typename R>
__host__ __device__ inline cplx<R> cmake(R a, R b) {
  cplx<R> c;
  c.x = a;
  c.y = b;
  return c;
}
template <typename R>
__host__ __device__ inline cplx<R> cadd(cplx<R> a, cplx<R> b) {
  return cmake<R>(a.x + b.x, a.y + b.y);
}
template <typename R>
__host__ __device__ inline cplx<R> csub(cplx<R> a, cplx<R> b) {
  return cmake<R>(a.x - b.x, a.y - b.y);
}
template <typename R>
__host__ __device__ inline cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return cmake<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename R>
__host__ __device__ inline cplx<R> cconj(cplx<R> a) {
  return cmake<R>(a.x, -a.y);
}
template <typename R>
__host__ __device__ inline cplx<R> cscale(cplx<R> a, R s) {
  return cmake<R>(a.x * s, a.y * s);
}

// FP64 complex helpers for plan-time device code
__host__ __device__ inline cplx<double> cexp_d(cplx<double> z) {
  double sn, cs;
  sincos(z.y, &sn, &cs);
  const double e = exp(z.x);
  return cmake<double>(e * cs, e * sn);
}

__host__ __device__ inline cplx<double> cdiv_d(cplx<double> a, cplx<double> b) {
  const double d = 1.0 / (b.x * b.x + b.y * b.y);
  return cmake<double>((a.x * b.x + a.y * b.y) * d, (a.y * b.x - a.x * b.y) * d);
}

// square root with Im <= 0 (and Re >= 0 on the real axis), computed without
// cancellation from the principal root
__host__ __device__ inline cplx<double> csqrt_im_nonpos_d(cplx<double> w) {
  const double a = hypot(w.x, w.y);
  if (a == 0.0) return cmake<double>(0.0, 0.0);
  double re, im;
  if (w.x >= 0.0) {
    re = sqrt(0.5 * (a + w.x));
    im = w.y / (2.0 * re);
  } else {
    im = copysign(sqrt(0.5 * (a - w.x)), w.y);
    re = w.y / (2.0 * im);
  }
  if (im > 0.0) {
    re = -re;
    im = -im;
  }
  return cmake<double>(re, im);
}


// Geometry of one uniform grid with an interpolation halo (Sec. 3.2, Eq. (grid)):
// node l on axis c sits at origin[c] + l h[c]; a point uses the q+1 nodes
// s..s+q.  Cells (boxes) are indexed by s in [0, nint].
struct GridGeom {
  int n[3];        // nodes per axis
  int nint[3];     // cells per axis
  int q;           // Lagrange degree
  double h[3];     // spacing
  double origin[3];
  double lo[3];    // start of the target region
};

// Lagrange basis value l_k(u) on the nodes 0..Q at position u.
template <int Q, typename R>
__host__ __device__ inline R lagrange_basis(int k, R u) {
  // c_k = 1 / prod_{j != k} (k - j) = (-1)^{Q-k} / (k! (Q-k)!)
  R num = R(1);
  R den = R(1);
#pragma unroll
  for (int j = 0; j <= Q; ++j) {
    if (j != k) {
      num *= (u - R(j));
      den *= R(k - j);
    }
  }
  return num / den;
}

// All Q+1 basis values at u.
template <int Q, typename R>
__host__ __device__ inline void lagrange_all(R u, R* w) {
  R left[Q + 1], right[Q + 1];
  left[0] = R(1);
#pragma unroll
  for (int k = 1; k <= Q; ++k) left[k] = left[k - 1] * (u - R(k - 1));
  right[Q] = R(1);
#pragma unroll
  for (int k = Q - 1; k >= 0; --k) right[k] = right[k + 1] * (u - R(k + 1));
  R fact = R(1);
  R inv_fact[Q + 1];
  inv_fact[0] = R(1);
#pragma unroll
  for (int k = 1; k <= Q; ++k) {
    fact *= R(k);
    inv_fact[k] = R(1) / fact;
  }
#pragma unroll
  for (int k = 0; k <= Q; ++k) {
    R c = inv_fact[k] * inv_fact[Q - k];
    if ((Q - k) & 1) c = -c;
    w[k] = c * left[k] * right[k];
  }
}

// 1 / prod_{j != k} (k - j) and prod_{j != k} (u - j): the two factors of the
// Lagrange basis value l_k(u) on the nodes 0..Q.
template <int Q>
__host__ __device__ inline double basis_den_inv(int k) {
  double d = 1.0;
#pragma unroll
  for (int j = 0; j <= Q; ++j)
    if (j != k) d *= static_cast<double>(k - j);
  return 1.0 / d;
}

template <int Q>
__host__ __device__ inline double basis_num(int k, double u) {
  double num = 1.0;
#pragma unroll
  for (int j = 0; j <= Q; ++j)
    if (j != k) num *= (u - static_cast<double>(j));
  return num;
}

// In-cell correction blocks (one per unordered pair of non-empty boxes).
// The pairs (B, B') of one box B are cut into lane groups: consecutive pairs
// whose columns fit one wavefront (a pair wider than 64 columns is cut into
// column chunks).  A group's blocks are stored row-interleaved (row r at
// voff + r * stride), and its columns map onto at most four runs of
// consecutive source points (boxes that follow each other in box order hold
// consecutive points after the box sort).
// Column-partial runs start on, and are padded to, whole 64-byte segments
// (kSymZAlign complex doubles): partial-segment writes cost a read-modify-write.
constexpr int kSymZAlign = 4;

struct alignas(16) SymGroup {
  int64_t voff;         // value of row 0, column 0
  int64_t zoff;         // column-partial slot of column 0 (columns contiguous)
  int32_t n0[4];        // first source point of each column run
  int32_t end[4];       // end column of each run (cumulative); unused runs: 64
  int32_t cum;          // columns (<= 64)
  int32_t stride;       // row stride of the values
  int32_t diag_lo, diag_hi;  // columns of the diagonal block B' = B (empty: lo == hi)
};

// Device pointers and sizes of the symmetric in-cell correction structure
// (mirrors the kernel-side SymArgs).
struct SymDev {
  int64_t npairs = 0, nitems = 0, nebox = 0, ngroups = 0, yslots = 0, zslots = 0;
  int max_box = 0;
  int32_t* ebox = nullptr;
  int32_t *pair_ebox_o = nullptr, *pair_ebox_s = nullptr;
  int64_t *pair_voff = nullptr, *pair_stride = nullptr;
  SymGroup* groups = nullptr;
  int32_t *item_ebox = nullptr, *item_order = nullptr;
  int64_t *item_gbeg = nullptr, *item_yoff = nullptr;
  int32_t* ebox_item_beg = nullptr;
  int64_t *in_ptr = nullptr, *in_base = nullptr;
};

// Geometry of the near-zone correction (Sec. 3.3 Step 4, Eq. (er)) as the
// fill, the tile builder and the position gradient traverse it.
struct CorrArgs {
  int nb[3], nint[3], per[3];
  int rc, id;
  int R, W;            // g0 table covers offsets [-R, R]^3, W = 2R + 1
  int64_t N;           // row points (observers)
  int64_t Nc;          // column points (sources; = N when the sets coincide)
  double L[3];
  double k0, k0_im;
  int nimg_axis;       // 2 id + 1
  const double* phase;    // device image phases (re, im), index (gx * A + gy) * A + gz, image g - id
  const double* phase_adj;  // conj(phase of image -i) at the index of image i (the C^H values)
  // per-axis candidate source boxes of an observer box S: entries
  // lent[c][loff[c][S] .. loff[c][S+1]) = b | (mask << 16), bit g of mask
  // marking image g - id (g = 0 only on non-periodic axes) as close
  const int32_t* loff[3];
  const int32_t* lent[3];
  int images_only;     // 1: drop the image-0 term (it is stored as symmetric blocks)
  // ball-shaped correction region: an offset d (boxes, image shift included)
  // is close when sum_c (d_c bw_c)^2 <= br2 (cube when ball == 0)
  int ball;
  double bw[3], br2;
};

// The ball test of the correction region, shared by host and device code.
__host__ __device__ inline bool ball_close(const double bw[3], double br2, int dx, int dy, int dz) {
  const double x = dx * bw[0], y = dy * bw[1], z = dz * bw[2];
  return x * x + y * y + z * z <= br2;
}

// The G0 table at near-grid node offsets ([W]^3 complex FP64) as the
// correction fill and gradient kernels read it: from global memory, or
// staged once per workgroup in LDS (real parts only for real kernels) when
// it fits kTabLdsBytes.
constexpr size_t kTabLdsBytes = 64 * 1024;
inline size_t tab_lds_bytes(int W, bool cplx) {
  return static_cast<size_t>(W) * W * W * (cplx ? 16 : 8);
}

#ifdef __HIPCC__
// Per-axis candidate source boxes of an observer box: entries (b | mask << 16)
// where bit (i + id) of mask marks image i_c as close.
__device__ inline void axis_range(const int32_t* __restrict__ off, int S, int& lo, int& hi) {
  lo = off[S];
  hi = off[S + 1];
}

// Whether image (imx, imy, imz) of the candidate source box (bx, by, bz) is
// close to the observer box S, given that it is close axis by axis (the
// per-axis masks hold the cube region): the image-0 term is left out when
// only images are stored, and the ball region also tests the whole offset.
__device__ inline bool image_close(const CorrArgs& a, const int S[3], int bx, int by, int bz, int imx, int imy,
                                   int imz) {
  if (a.images_only && imx == 0 && imy == 0 && imz == 0) return false;
  return !a.ball || ball_close(a.bw, a.br2, S[0] - bx - imx * a.nint[0], S[1] - by - imy * a.nint[1],
                               S[2] - bz - imz * a.nint[2]);
}

// Whether any image of the candidate source box is close (the per-axis masks
// mx, my, mz: bit g marks image g - id on that axis as close axis by axis).
__device__ inline bool any_close(const CorrArgs& a, const int S[3], int bx, int by, int bz, int mx, int my, int mz) {
  const int A = a.nimg_axis;
  for (int gx = 0; gx < A; ++gx) {
    if (!((mx >> gx) & 1)) continue;
    for (int gy = 0; gy < A; ++gy) {
      if (!((my >> gy) & 1)) continue;
      for (int gz = 0; gz < A; ++gz) {
        if (!((mz >> gz) & 1)) continue;
        if (image_close(a, S, bx, by, bz, gx - a.id * a.per[0], gy - a.id * a.per[1], gz - a.id * a.per[2]))
          return true;
      }
    }
  }
  return false;
}

// Wave-level inclusive prefix sum and total of an int, and sum of a double.
__device__ inline int wave_incl_scan(int v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Orders one wavefront's LDS writes before its later reads (and reads before
// later writes): the lanes of a wave run in lockstep, so a compiler and
// memory fence at workgroup scope is all that is needed.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

constexpr int kPairBPL = 2;                    // candidate boxes per lane per chunk
constexpr int kPairCH = 64 * kPairBPL;         // candidate boxes per chunk
constexpr int kPairListInts = 3 * kPairCH + 1;  // per-wave LDS lists (prefix, first point, candidate)

// The close pairs of one row point, enumerated by one wavefront: the row's
// box S has per-axis candidate lists [lo, hi) of column boxes; their product
// is taken kPairCH candidates at a time, every lane counting the points of
// kPairBPL boxes (zero for boxes with no close image), a wave prefix sum
// laying the chunk's pairs out, and the pairs are then handed out 64 at a
// time, one per lane (lane t finds its box by binary search over the
// prefix).  Pairs come in candidate order (x, then y, then z box), points in
// order within a box: body(t, n, bx, by, bz, mx, my, mz) runs on the lanes
// that hold pair t of the row (t counted from 0 over the whole row), n being
// the column point and m* the per-axis image masks.  lists: kPairListInts
// ints of LDS owned by the wave.
template <typename F>
__device__ inline void wave_pairs(const CorrArgs& a, const int S[3], const int lo[3], const int hi[3],
                                  const int32_t* __restrict__ box_start, int* lists, int lane, F&& body) {
  int* pre = lists;              // [kPairCH + 1] pair offsets of the chunk's boxes
  int* cn0 = pre + kPairCH + 1;  // [kPairCH] first point of each box
  int* ccd = cn0 + kPairCH;      // [kPairCH] candidate index of each box
  const int Ly = hi[1] - lo[1], Lz = hi[2] - lo[2];
  const int ncand = (hi[0] - lo[0]) * Ly * Lz;
  int64_t tbase = 0;
  for (int c0 = 0; c0 < ncand; c0 += kPairCH) {
    int cnt[kPairBPL], n0[kPairBPL];
    int sum = 0;
#pragma unroll
    for (int i = 0; i < kPairBPL; ++i) {
      const int c = c0 + lane * kPairBPL + i;
      cnt[i] = 0;
      n0[i] = 0;
      if (c < ncand) {
        const int ex = a.lent[0][lo[0] + c / (Ly * Lz)], ey = a.lent[1][lo[1] + (c / Lz) % Ly],
                  ez = a.lent[2][lo[2] + c % Lz];
        const int bx = ex & 0xffff, by = ey & 0xffff, bz = ez & 0xffff;
        if (any_close(a, S, bx, by, bz, ex >> 16, ey >> 16, ez >> 16)) {
          const int64_t b = (static_cast<int64_t>(bx) * a.nb[1] + by) * a.nb[2] + bz;
          n0[i] = box_start[b];
          cnt[i] = box_start[b + 1] - n0[i];
        }
      }
      sum += cnt[i];
    }
    const int incl = wave_incl_scan(sum, lane);
    const int tot = __shfl(incl, 63, 64);
    int run = incl - sum;
#pragma unroll
    for (int i = 0; i < kPairBPL; ++i) {
      pre[lane * kPairBPL + i] = run;
      cn0[lane * kPairBPL + i] = n0[i];
      ccd[lane * kPairBPL + i] = c0 + lane * kPairBPL + i;
      run += cnt[i];
    }
    if (lane == 0) pre[kPairCH] = tot;
    wave_lds_sync();
    for (int t0 = 0; t0 < tot; t0 += 64) {
      const int t = t0 + lane;
      if (t < tot) {
        // the box holding pair t: the largest i with pre[i] <= t (it has at
        // least one point since pre[i + 1] > t)
        int ilo = 0, ihi = kPairCH - 1;
        while (ilo < ihi) {
          const int mid = (ilo + ihi + 1) >> 1;
          if (pre[mid] <= t) ilo = mid;
          else ihi = mid - 1;
        }
        const int n = cn0[ilo] + (t - pre[ilo]);
        const int c = ccd[ilo];
        const int ex = a.lent[0][lo[0] + c / (Ly * Lz)], ey = a.lent[1][lo[1] + (c / Lz) % Ly],
                  ez = a.lent[2][lo[2] + c % Lz];
        body(tbase + t, n, ex & 0xffff, ey & 0xffff, ez & 0xffff, ex >> 16, ey >> 16, ez >> 16);
      }
    }
    tbase += tot;
    wave_lds_sync();
  }
}

template <bool CPLX>
__device__ inline void tab_stage(const cplx<double>* __restrict__ g, double* lt, int64_t n) {
  for (int64_t t = threadIdx.x; t < n; t += blockDim.x) {
    const cplx<double> v = g[t];
    if (CPLX) {
      lt[2 * t] = v.x;
      lt[2 * t + 1] = v.y;
    } else {
      lt[t] = v.x;
    }
  }
  __syncthreads();
}

template <bool CPLX, bool LT>
__device__ inline void tab_get(const cplx<double>* __restrict__ g, const double* lt, int64_t i, double& x,
                               double& y) {
  if constexpr (LT) {
    if constexpr (CPLX) {
      typedef double d2_t __attribute__((ext_vector_type(2)));
      const d2_t v = reinterpret_cast<const d2_t*>(lt)[i];
      x = v.x;
      y = v.y;
    } else {
      x = lt[i];
      y = 0.0;
    }
  } else {
    const cplx<double> t = g[i];
    x = t.x;
    y = CPLX ? t.y : 0.0;
  }
}
#endif

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace fftpim

// Work arrays of one near-grid + far-zone pass (all planes-innermost).
struct WorkSet {
  void* grid0 = nullptr;     // [nx][ny][nz][planes] near grid
  void* bufA = nullptr;      // [nx][ny][Mz][planes] after the z pass
  void* bufB = nullptr;      // [nx][My][Mz][planes] after the y pass
  void* far_mom = nullptr;   // [far boxes][(qf+1)^3][planes] box moments
  void* far_q = nullptr;     // [Ngf][planes] far source grid
  void* far_u = nullptr;     // [Ngf][planes] far observer grid
  void* far_part = nullptr;  // [splits][Ngf][planes] partial grid sums (direct far sum)
  void* far_bufA = nullptr;  // [nfx][nfy][Mfz][planes] after the z pass (FFT far sum)
  void* far_bufB = nullptr;  // [nfx][Mfy][Mfz][planes] after the y pass (FFT far sum)
};

// Arrays of the fused forward + adjoint pair beyond the plan's own workspace:
// a second work set, the packed adjoint input and the three parts of A^H v.
struct PairBufs {
  WorkSet ws2;
  void* v_int = nullptr;
  void* u_int2 = nullptr;
  void* u_corr2 = nullptr;
  void* u_far2 = nullptr;
};

struct fftpim_plan_s {
  fftpim::Lattice lat;
  fftpim_problem_t problem;
  fftpim_params_t prm;
  int64_t N = 0;               // sources
  // separate observers (otherwise the observer arrays below alias the
  // source arrays and No = N)
  bool sep = false;
  int64_t No = 0;
  int32_t* perm_o = nullptr;      // observer plan position -> caller index
  int32_t* near_s_o = nullptr;    // observer near stencils, weights, box sort
  double* near_u_o = nullptr;
  double* near_w_o = nullptr;
  int32_t* box_start_o = nullptr;
  // conjugate-transpose correction with separate observers: CSR with source
  // rows and observer columns holding C^H
  int64_t* rowptr_a = nullptr;
  int32_t* col_a = nullptr;
  void* val_a = nullptr;
  int32_t* corr_order_a = nullptr;
  int64_t corr_slots_a = 0;
  int64_t nnz_a = 0;
  int device = 0;              // HIP device current when the plan was made
  bool complex_kernel = true;  // G0 or the phases are complex
  bool nonhermitian = false;   // k0 != 0 or a complex phase shift: C^H needs its own values
  std::complex<double> self_coef = 0.0;  // lim_{r->0}[G^p - G0] (self_mode exclude)

  // near grid
  fftpim::GridGeom ng;
  int M[3];        // FFT sizes (2 n)
  int nb[3];       // boxes per axis (nint + 1)
  // far grids (source grid origin; the observer grid is shifted by -h/2)
  fftpim::GridGeom fg;
  int fnb[3];

  // sorted geometry (device)
  int32_t* perm = nullptr;        // plan position -> caller index
  int32_t* near_s = nullptr;      // [3][N] stencil starts (= near boxes)
  double* near_u = nullptr;       // [3][N] position within the stencil
  double* near_w = nullptr;       // [3][q+1][N] 1D Lagrange weights
  double* fs_w = nullptr;         // [3][qf+1][N] far source-grid weights
  double* fo_w = nullptr;         // [3][qf+1][N] far observer-grid weights
  int32_t* box_start = nullptr;   // [nb^3 + 1] first point of each box
  int32_t* fs_s = nullptr;        // far source-grid stencils [3][N]
  double* fs_u = nullptr;
  int32_t* fo_s = nullptr;        // far observer-grid stencils [3][N]
  double* fo_u = nullptr;
  int32_t* fperm_s = nullptr;     // points ordered by far source box
  int32_t* fbox_start_s = nullptr;
  int32_t* fperm_o = nullptr;     // points ordered by far observer box
  int32_t* fbox_start_o = nullptr;
  int fmax_box_s = 0, fmax_box_o = 0;  // most points in one far box (source / observer grid)

  // tables
  void* near_hat = nullptr;       // [Mx][My][Mz] complex R, scaled by 1/(Mx My Mz)
  void* twiddle[3] = {nullptr, nullptr, nullptr};  // per axis, M/2 complex R
  void* far_table = nullptr;      // [(2nf-1)^3] complex R (direct far sum)
  bool far_fft = false;           // far grid sum as a zero-padded FFT convolution
  int Mf[3] = {0, 0, 0};          // its transform lengths
  void* far_hat = nullptr;        // [Mfx][Mfy][Mfz] complex R, scaled by 1/(Mfx Mfy Mfz)
  void* ftwiddle[3] = {nullptr, nullptr, nullptr};

  // in-cell correction as symmetric box-pair blocks (when sym is set), the
  // CSR below then holds only the close-image part
  bool sym = false;
  fftpim::SymDev symd;
  void* sym_vals = nullptr;
  int64_t sym_nvals = 0;
  void* sym_ypart = nullptr;      // [item slots][planes] complex double
  void* sym_zpart = nullptr;      // [pair slots][planes] complex double

  // correction (FP64 values)
  int64_t* rowptr = nullptr;
  double* sums_work = nullptr;     // scratch of the plane sums
  // node-major transposed near weights (plans with at most kSpreadCsrPlanes
  // planes), over the nodes that have entries (wt_node) only
  int64_t* wt_node = nullptr;
  int64_t wt_nnodes = 0;
  int64_t* wt_row = nullptr;
  int32_t* wt_idx = nullptr;
  double* wt_val = nullptr;
  int32_t* corr_order = nullptr;   // [corr_slots] row of each wavefront slot (-1: idle)
  // dense row tiles (real correction values): see build_tiles
  bool tile = false;
  int64_t ntiles = 0, tile_nvals = 0;
  int32_t* tile_rows = nullptr;    // [ntiles * 16] observers (-1: padding)
  int64_t* tile_coff = nullptr;    // [ntiles + 1] union column ranges
  int32_t* tile_cols = nullptr;    // union columns, ascending per tile
  int64_t* tile_voff = nullptr;    // [ntiles + 1] value ranges (64 per k-step)
  double* tile_vals = nullptr;
  int64_t corr_slots = 0;
  int32_t* col = nullptr;
  void* val = nullptr;            // double or complex double
  void* val_adj = nullptr;        // Helmholtz only: values of C^H on the same pattern
  int64_t nnz = 0;
  // position gradient: the correction traversal of the fill (all images),
  // the G0 table at node offsets, the sorted positions [3][N], and a [N][3]
  // accumulator made on the first gradient call
  fftpim::CorrArgs grad_ca{};
  void* g0tab = nullptr;
  double* pos3 = nullptr;
  double* grad_acc = nullptr;

  // workspace
  int nplanes_max = 0;
  void* q_int = nullptr;          // [N][planes] complex R (plan order)
  void* u_int = nullptr;          // [N][planes] complex R: near-grid part
  void* u_corr = nullptr;         // [N][planes] correction part
  void* u_far = nullptr;          // [N][planes] far-zone part
  // the correction and the far zone run on their own streams, forked from and
  // joined back into the caller's stream with events (default priority)
  hipStream_t s_corr = nullptr, s_far = nullptr, s_near = nullptr;
  hipEvent_t ev_fork = nullptr, ev_corr = nullptr, ev_far = nullptr, ev_near = nullptr;
  WorkSet ws;                     // near-grid and far-zone work arrays
  PairBufs pair;                  // fused pair only, made on its first call
  double* sums = nullptr;         // [2][planes] neutrality / mean sums
  int* status_dev = nullptr;      // latched device-detected error

  // stage timing (fftpim_stage_times)
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, size_t>> ev_pairs;  // (stage, index of the start event)
  double stage_ms[8] = {0};
  int64_t stage_calls[8] = {0};

  std::vector<fftpim::DevBuf> allocations;
  int64_t device_bytes = 0;
  double plan_seconds = 0.0;
  hipStream_t last_stream = nullptr;
};
