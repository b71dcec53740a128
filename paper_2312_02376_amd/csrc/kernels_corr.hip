// Near-zone error correction, Sec. 3.3 Step 4, Eq. (er), with only the close
// images kept (end of Sec. 3.3).
//
// For an observer m and a source n, the image i (|i_c| <= i_d on periodic
// axes) is close when the box offset d = s_m - s_n - i * nint lies in the
// correction region: the cube max_c |d_c| <= r_c, or the ball
// sum_c (d_c h_c / h_max)^2 <= r^2 of Eq. (er).  The stored entry is
//     C[m, n] = sum_{close i} phi_i X_i(m, n),
//     X_i(m, n) = G0(r_m - r_n - R_i) - G_grid,i(m, n)      (G0 term dropped
//                                                            for n = m, i = 0)
//     G_grid,i(m, n) = sum_a sum_b w_a(r_m) w_b(r_n) G0tab((a - b - i nint) h)
// and the double sum over the two (q+1)^3 stencils is evaluated through the
// 1D weight correlations C_c(d) = sum_{a - b = d} w_a w_b, d in [-q, q]:
//     G_grid,i = sum_{d in [-q, q]^3} Cx(dx) Cy(dy) Cz(dz) G0tab(Delta + d),
// Delta = s_m - s_n - i nint.  Values are FP64.  For a Helmholtz kernel a
// second array on the same (symmetric) pattern holds the conjugate transpose:
// entry (n, m) of C^H equals sum_{close i} phi_i conj(X_i(n, m)).
#include "kernels.h"

namespace fftpim {


__global__ void k_corr_count(CorrArgs a, const int32_t* __restrict__ s3, const int32_t* __restrict__ box_start,
                             int64_t* __restrict__ rowcount) {
  const int32_t *loff0 = a.loff[0], *loff1 = a.loff[1], *loff2 = a.loff[2];
  const int32_t *lent0 = a.lent[0], *lent1 = a.lent[1], *lent2 = a.lent[2];
  int64_t m = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (m >= a.N) return;
  int x0, x1, y0, y1, z0, z1;
  const int S[3] = {s3[m], s3[a.N + m], s3[2 * a.N + m]};
  axis_range(loff0, S[0], x0, x1);
  axis_range(loff1, S[1], y0, y1);
  axis_range(loff2, S[2], z0, z1);
  int64_t cnt = 0;
  for (int ix = x0; ix < x1; ++ix) {
    int bx = lent0[ix] & 0xffff;
    for (int iy = y0; iy < y1; ++iy) {
      int by = lent1[iy] & 0xffff;
      for (int iz = z0; iz < z1; ++iz) {
        int bz = lent2[iz] & 0xffff;
        // no close image left (e.g. only the image-0 term, which lives in the
        // symmetric blocks, or none inside the ball)
        if (!any_close(a, S, bx, by, bz, lent0[ix] >> 16, lent1[iy] >> 16, lent2[iz] >> 16)) continue;
        int64_t b = (static_cast<int64_t>(bx) * a.nb[1] + by) * a.nb[2] + bz;
        cnt += box_start[b + 1] - box_start[b];
      }
    }
  }
  rowcount[m] = cnt;
}

// The correction values of Eq. (er): for each close triple (m, n, i),
// phi_i [G0(r_m - r_n - R_i) - sum_ab w_a(r_m) w_b(r_n) G0tab(a - b + D_i)],
// the double sum taken through 1D weight correlations.  Rows are the points
// of s3/u3/pos3 ([3][N]), columns those of box_start/u3c/pos3c ([3][Nc]);
// the two sets coincide unless the plan has separate observers.  A pair at
// zero distance (the self pair, or an observer placed on a source) keeps
// only its grid part.  One wavefront per row (kFillRPW rows in turn):
// wave_pairs hands the row's close pairs to the lanes 64 at a time in the
// order the count kernel and the row pointers assume, so entry t of row m
// goes to rowptr[m] + t.  ADJ also writes the values of C^H on the same
// pattern.  The G0 table is read from LDS when LT.
constexpr int kFillWaves = 4, kFillRPW = 8;

inline size_t fill_list_bytes() { return static_cast<size_t>(kFillWaves) * kPairListInts * sizeof(int); }

template <int Q, bool CPLX, bool ADJ, bool LT>
__global__ void __launch_bounds__(64 * kFillWaves) k_corr_fill_wave(
    CorrArgs a, const int32_t* __restrict__ s3, const double* __restrict__ u3, const double* __restrict__ pos3,
    const double* __restrict__ u3c, const double* __restrict__ pos3c, const int32_t* __restrict__ box_start,
    const cplx<double>* __restrict__ g0tab, const int64_t* __restrict__ rowptr, int32_t* __restrict__ col,
    void* __restrict__ val_v, void* __restrict__ vadj_v) {
  extern __shared__ __align__(16) double lt[];
  const int64_t tabn = static_cast<int64_t>(a.W) * a.W * a.W;
  if (LT) tab_stage<CPLX>(g0tab, lt, tabn);
  int* lists = reinterpret_cast<int*>(lt + (LT ? tabn * (CPLX ? 2 : 1) : 0));
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
  const int lane = static_cast<int>(threadIdx.x) & 63;
  int* wl = lists + wave * kPairListInts;
  const int64_t N = a.N, Nc = a.Nc;
  const int A = a.nimg_axis, W = a.W, R = a.R;
  double* valr = static_cast<double*>(val_v);
  cplx<double>* valc = static_cast<cplx<double>*>(val_v);
  cplx<double>* vadj = static_cast<cplx<double>*>(vadj_v);
  for (int rr = 0; rr < kFillRPW; ++rr) {
    const int64_t m = (static_cast<int64_t>(blockIdx.x) * kFillWaves + wave) * kFillRPW + rr;
    if (m >= N) break;
    const int S[3] = {s3[m], s3[N + m], s3[2 * N + m]};
    double wm[3][Q + 1];
#pragma unroll
    for (int c = 0; c < 3; ++c) lagrange_all<Q, double>(u3[c * N + m], wm[c]);
    const double rm[3] = {pos3[m], pos3[N + m], pos3[2 * N + m]};
    int lo[3], hi[3];
    axis_range(a.loff[0], S[0], lo[0], hi[0]);
    axis_range(a.loff[1], S[1], lo[1], hi[1]);
    axis_range(a.loff[2], S[2], lo[2], hi[2]);
    const int64_t j0 = rowptr[m];
    wave_pairs(a, S, lo, hi, box_start, wl, lane, [&](int64_t t, int n, int bx, int by, int bz, int mx, int my, int mz) {
      double wn[3][Q + 1];
#pragma unroll
      for (int c = 0; c < 3; ++c) lagrange_all<Q, double>(u3c[c * Nc + n], wn[c]);
      double C[3][2 * Q + 1];
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int d = -Q; d <= Q; ++d) {
          double sw = 0.0;
#pragma unroll
          for (int aa = 0; aa <= Q; ++aa) {
            if (aa - d < 0 || aa - d > Q) continue;
            sw += wm[c][aa] * wn[c][aa - d];
          }
          C[c][d + Q] = sw;
        }
      const double rn[3] = {pos3c[n], pos3c[Nc + n], pos3c[2 * Nc + n]};
      double fr = 0.0, fi = 0.0, ar = 0.0, ai = 0.0;
      for (int gx = 0; gx < A; ++gx) {
        if (!((mx >> gx) & 1)) continue;
        const int imx = gx - a.id * a.per[0];
        for (int gy = 0; gy < A; ++gy) {
          if (!((my >> gy) & 1)) continue;
          const int imy = gy - a.id * a.per[1];
          for (int gz = 0; gz < A; ++gz) {
            if (!((mz >> gz) & 1)) continue;
            const int imz = gz - a.id * a.per[2];
            if (!image_close(a, S, bx, by, bz, imx, imy, imz)) continue;
            const int D[3] = {S[0] - bx - imx * a.nint[0], S[1] - by - imy * a.nint[1], S[2] - bz - imz * a.nint[2]};
            // exact part (a pair at zero distance keeps only its grid part)
            double er = 0.0, ei = 0.0;
            const double ddx = rm[0] - rn[0] - imx * a.L[0];
            const double ddy = rm[1] - rn[1] - imy * a.L[1];
            const double ddz = rm[2] - rn[2] - imz * a.L[2];
            const double r = sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
            if (r > 0.0) {
              const double inv = (a.k0_im != 0.0 ? exp(a.k0_im * r) : 1.0) / (4.0 * M_PI * r);
              if (CPLX) {
                double sn, cs;
                sincos(a.k0 * r, &sn, &cs);
                er = cs * inv;
                ei = -sn * inv;
              } else {
                er = inv;
              }
            }
            // grid part: x stays a loop (bounding the registers), its weight
            // picked by selects so C stays in registers
            double gr = 0.0, gi = 0.0;
#pragma nounroll
            for (int dx = -Q; dx <= Q; ++dx) {
              double cx = 0.0;
#pragma unroll
              for (int u = 0; u <= 2 * Q; ++u) cx = (u == dx + Q) ? C[0][u] : cx;
              const int64_t rowx = static_cast<int64_t>(D[0] + dx + R) * W;
#pragma unroll
              for (int dy = -Q; dy <= Q; ++dy) {
                const double cxy = cx * C[1][dy + Q];
                const int64_t toff = (rowx + D[1] + dy + R) * W + (D[2] + R);
                double sr = 0.0, si = 0.0;
#pragma unroll
                for (int dz = -Q; dz <= Q; ++dz) {
                  double tx, ty;
                  tab_get<CPLX, LT>(g0tab, lt, toff + dz, tx, ty);
                  sr += C[2][dz + Q] * tx;
                  if (CPLX) si += C[2][dz + Q] * ty;
                }
                gr += cxy * sr;
                gi += cxy * si;
              }
            }
            const double xr = er - gr, xi = ei - gi;
            if (CPLX) {
              const int pidx = (gx * A + gy) * A + gz;
              const double pr = a.phase[2 * pidx], pi = a.phase[2 * pidx + 1];
              fr += pr * xr - pi * xi;
              fi += pr * xi + pi * xr;
              if (ADJ) {
                // entry (m, n) of C^H: psi_i conj(X), psi_i = conj(phase_{-i})
                const double qr = a.phase_adj[2 * pidx], qi = a.phase_adj[2 * pidx + 1];
                ar += qr * xr + qi * xi;
                ai += qi * xr - qr * xi;
              }
            } else {
              fr += xr;
            }
          }
        }
      }
      const int64_t j = j0 + t;
      col[j] = n;
      if (CPLX) {
        valc[j] = cmake<double>(fr, fi);
        if (ADJ) vadj[j] = cmake<double>(ar, ai);
      } else {
        valr[j] = fr;
      }
    });
  }
}

// Writes (does not accumulate) the correction of every row.
// One wavefront per row; lanes stride over the row two entries at a time
// (independent accumulators keep more loads in flight); the column and value
// streams are read once, so they are loaded non-temporally and leave the
// cache to the gathered amplitudes.  Wave-level reduction at the end.
typedef double dbl2_t __attribute__((ext_vector_type(2)));

template <bool CPLX>
__device__ inline void load_val(const void* __restrict__ val_v, int64_t j, double& vr, double& vi) {
  if (CPLX) {
    const dbl2_t v = __builtin_nontemporal_load(static_cast<const dbl2_t*>(val_v) + j);
    vr = v.x;
    vi = v.y;
  } else {
    vr = __builtin_nontemporal_load(static_cast<const double*>(val_v) + j);
    vi = 0.0;
  }
}

template <typename R, bool CPLX, int PB>
__global__ void __launch_bounds__(256) k_corr_spmv(const int64_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ col,
                                                   const void* __restrict__ val_v, int64_t N,
                                                   const int32_t* __restrict__ order,
                                                   const cplx<R>* __restrict__ qint, int P,
                                                   cplx<R>* __restrict__ uint, int accumulate) {
  const int lane = threadIdx.x & 63;
  const int64_t slot = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t row = order != nullptr ? order[slot] : slot;
  if (row < 0 || row >= N) return;
  const int p0 = blockIdx.y * PB;
  double ar[PB], ai[PB], br[PB], bi[PB];
#pragma unroll
  for (int pp = 0; pp < PB; ++pp) ar[pp] = ai[pp] = br[pp] = bi[pp] = 0.0;
  const int64_t j1 = rowptr[row + 1];
  int64_t j = rowptr[row] + lane;
  for (; j + 64 < j1; j += 128) {
    const int n0 = __builtin_nontemporal_load(col + j);
    const int n1 = __builtin_nontemporal_load(col + j + 64);
    double v0r, v0i, v1r, v1i;
    load_val<CPLX>(val_v, j, v0r, v0i);
    load_val<CPLX>(val_v, j + 64, v1r, v1i);
#pragma unroll
    for (int pp = 0; pp < PB; ++pp) {
      if (p0 + pp < P) {
        const cplx<R> q0 = qint[static_cast<int64_t>(n0) * P + p0 + pp];
        const cplx<R> q1 = qint[static_cast<int64_t>(n1) * P + p0 + pp];
        const double q0r = static_cast<double>(q0.x), q0i = static_cast<double>(q0.y);
        const double q1r = static_cast<double>(q1.x), q1i = static_cast<double>(q1.y);
        ar[pp] += v0r * q0r - v0i * q0i;
        ai[pp] += v0r * q0i + v0i * q0r;
        br[pp] += v1r * q1r - v1i * q1i;
        bi[pp] += v1r * q1i + v1i * q1r;
      }
    }
  }
  if (j < j1) {
    const int n0 = __builtin_nontemporal_load(col + j);
    double v0r, v0i;
    load_val<CPLX>(val_v, j, v0r, v0i);
#pragma unroll
    for (int pp = 0; pp < PB; ++pp) {
      if (p0 + pp < P) {
        const cplx<R> q0 = qint[static_cast<int64_t>(n0) * P + p0 + pp];
        const double q0r = static_cast<double>(q0.x), q0i = static_cast<double>(q0.y);
        ar[pp] += v0r * q0r - v0i * q0i;
        ai[pp] += v0r * q0i + v0i * q0r;
      }
    }
  }
#pragma unroll
  for (int pp = 0; pp < PB; ++pp) {
    ar[pp] += br[pp];
    ai[pp] += bi[pp];
    for (int off = 32; off > 0; off >>= 1) {
      ar[pp] += __shfl_down(ar[pp], off, 64);
      ai[pp] += __shfl_down(ai[pp], off, 64);
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int pp = 0; pp < PB; ++pp) {
      if (p0 + pp < P) {
        cplx<R> o = cmake<R>(static_cast<R>(ar[pp]), static_cast<R>(ai[pp]));
        if (accumulate) {
          const cplx<R> prev = uint[row * P + p0 + pp];
          o = cmake<R>(static_cast<R>(static_cast<double>(prev.x) + ar[pp]),
                       static_cast<R>(static_cast<double>(prev.y) + ai[pp]));
        }
        uint[row * P + p0 + pp] = o;
      }
    }
  }
}

// Many right-hand sides: the 64 lanes of a wavefront cover LP planes x
// (64 / LP) entries of one row, so every CSR entry is read once per row and
// the amplitudes of one source are one contiguous, coalesced load.  Four
// entries per lane slot are in flight at once.  Partial sums over the entry
// slots are combined with lane shuffles in a fixed order.
template <typename R, bool CPLX, int LP>
__global__ void __launch_bounds__(256) k_corr_spmm(const int64_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ col,
                                                   const void* __restrict__ val_v, int64_t N,
                                                   const int32_t* __restrict__ order,
                                                   const cplx<R>* __restrict__ qint, int P,
                                                   cplx<R>* __restrict__ uint, int accumulate) {
  constexpr int E = 64 / LP;
  constexpr int U = 4;
  const int lane = threadIdx.x & 63;
  const int e = lane / LP, pl = lane % LP;
  const int64_t slot = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t row = order != nullptr ? order[slot] : slot;
  if (row < 0 || row >= N) return;
  const int64_t j0 = rowptr[row], j1 = rowptr[row + 1];
  for (int pc = 0; pc < P; pc += LP) {
    const int p = pc + pl;
    const bool pok = p < P;
    double ar = 0.0, ai = 0.0;
    int64_t j = j0 + e;
    for (; j + (U - 1) * E < j1; j += U * E) {
      int n[U];
      double vr[U], vi[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        n[u] = __builtin_nontemporal_load(col + j + u * E);
        load_val<CPLX>(val_v, j + u * E, vr[u], vi[u]);
      }
      if (pok) {
        cplx<R> q[U];
#pragma unroll
        for (int u = 0; u < U; ++u) q[u] = qint[static_cast<int64_t>(n[u]) * P + p];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const double qr = static_cast<double>(q[u].x), qi = static_cast<double>(q[u].y);
          ar += vr[u] * qr - vi[u] * qi;
          ai += vr[u] * qi + vi[u] * qr;
        }
      }
    }
    for (; j < j1; j += E) {
      const int n = col[j];
      double vr, vi;
      load_val<CPLX>(val_v, j, vr, vi);
      if (pok) {
        const cplx<R> q = qint[static_cast<int64_t>(n) * P + p];
        const double qr = static_cast<double>(q.x), qi = static_cast<double>(q.y);
        ar += vr * qr - vi * qi;
        ai += vr * qi + vi * qr;
      }
    }
    for (int off = LP; off < 64; off <<= 1) {
      ar += __shfl_xor(ar, off, 64);
      ai += __shfl_xor(ai, off, 64);
    }
    if (e == 0 && pok) {
      cplx<R> o = cmake<R>(static_cast<R>(ar), static_cast<R>(ai));
      if (accumulate) {
        const cplx<R> prev = uint[row * P + p];
        o = cmake<R>(static_cast<R>(static_cast<double>(prev.x) + ar), static_cast<R>(static_cast<double>(prev.y) + ai));
      }
      uint[row * P + p] = o;
    }
  }
}

// ---------------------------------------------------------------------------
// Dense row tiles (real correction values): 16 observers x the union of their
// corrected sources, zeros where a pair is not corrected.  A tile's values are
// stored in MFMA A-fragment order: k-step s holds 64 doubles, lane l = r +
// 16 kk giving row r, tile column 4 s + kk.
// ---------------------------------------------------------------------------

// Plan time: scatter each observer's CSR entries into its tile (one thread
// per observer, so repeated columns of several images add up without races).
__global__ void k_tile_fill(const int32_t* __restrict__ tile_rows, int64_t nslots, const int64_t* __restrict__ rowptr,
                            const int32_t* __restrict__ col, const double* __restrict__ val,
                            const int64_t* __restrict__ coff, const int32_t* __restrict__ cols,
                            const int64_t* __restrict__ voff, double* __restrict__ tv) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= nslots) return;
  const int m = tile_rows[idx];
  if (m < 0) return;
  const int64_t t = idx >> 4;
  const int r = static_cast<int>(idx & 15);
  const int64_t c0 = coff[t], C = coff[t + 1] - c0;
  for (int64_t j = rowptr[m]; j < rowptr[m + 1]; ++j) {
    const int n = col[j];
    int64_t lo = 0, hi = C - 1;  // the column is in the tile's sorted list
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (cols[c0 + mid] < n) lo = mid + 1; else hi = mid;
    }
    tv[voff[t] + (lo >> 2) * 64 + r + 16 * (lo & 3)] += val[j];
  }
}

// Apply: one wavefront per tile.  The tile's real-column view of the
// amplitudes ([N][2P] reals, re/im interleaved) is taken 64 columns at a time
// as four 16-column MFMA chunks; each k-step gathers four source rows (one per
// lane group) and runs four 16x16x4 FP64 MFMAs with the same value fragment.
// FP64 accumulator element r of lane l holds row 4 r + l / 16, column l % 16.
typedef double tile_d4 __attribute__((ext_vector_type(4)));
constexpr int kTileWaves = 4;

template <typename R>
// six waves per SIMD (register budget) hide the gather latency better than four
__global__ void __launch_bounds__(64 * kTileWaves) __attribute__((amdgpu_waves_per_eu(6, 8))) k_corr_tile(const int32_t* __restrict__ tile_rows, int64_t ntiles,
                                                               const int64_t* __restrict__ coff,
                                                               const int32_t* __restrict__ cols,
                                                               const int64_t* __restrict__ voff,
                                                               const double* __restrict__ tv,
                                                               const R* __restrict__ x, int P2, R* __restrict__ u) {
  const int lane = threadIdx.x & 63;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kTileWaves + (threadIdx.x >> 6);
  if (t >= ntiles) return;
  const int64_t c0 = coff[t], C = coff[t + 1] - c0;
  const int64_t nks = (C + 3) >> 2;
  const double* v = tv + voff[t];
  const int kk = lane >> 4, jl = lane & 15;
  for (int cg = 0; cg < P2; cg += 64) {
    tile_d4 acc[4];
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) acc[ch] = tile_d4{0.0, 0.0, 0.0, 0.0};
    // 64 union columns (16 k-steps) at a time: each lane loads one column
    // index and the k-steps take theirs by lane shuffle.  Loads run one group
    // of two k-steps ahead of the MFMAs (software pipelining); they are
    // branch-free (idle slots read valid addresses and are zeroed), so the
    // compiler keeps the next group's loads in flight across the MFMAs.
    constexpr int U = 2;
    for (int64_t cb = 0; cb < C; cb += 64) {
      const int colv = (cb + lane < C) ? cols[c0 + cb + lane] : -1;
      const int64_t sb = cb >> 2;
      const int ns = static_cast<int>(min<int64_t>(16, nks - sb));
      auto load_group = [&](int s0, double (&a)[U], R (&b)[U][4]) {
#pragma unroll
        for (int uu = 0; uu < U; ++uu) {
          const int s = s0 + uu;
          const bool sok = s < ns;
          const double av = __builtin_nontemporal_load(v + (sb + (sok ? s : 0)) * 64 + lane);
          a[uu] = sok ? av : 0.0;
          const int n = __shfl(colv, (4 * s + kk) & 63, 64);
          const bool nok = sok && n >= 0;
#pragma unroll
          for (int ch = 0; ch < 4; ++ch) {
            const int j = cg + 16 * ch + jl;
            const bool ok = nok && j < P2;
            const R xv = x[static_cast<int64_t>(ok ? n : 0) * P2 + (ok ? j : 0)];
            b[uu][ch] = ok ? xv : R(0);
          }
        }
      };
      double a0[U];
      R b0[U][4];
      load_group(0, a0, b0);
      for (int s0 = 0; s0 < ns; s0 += U) {
        double a1[U];
        R b1[U][4];
        load_group(s0 + U, a1, b1);  // past the end: zeros from valid addresses
#pragma unroll
        for (int uu = 0; uu < U; ++uu)
#pragma unroll
          for (int ch = 0; ch < 4; ++ch)
            acc[ch] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[uu], static_cast<double>(b0[uu][ch]), acc[ch], 0, 0, 0);
#pragma unroll
        for (int uu = 0; uu < U; ++uu) {
          a0[uu] = a1[uu];
#pragma unroll
          for (int ch = 0; ch < 4; ++ch) b0[uu][ch] = b1[uu][ch];
        }
      }
    }
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
      const int j = cg + 16 * ch + jl;
      if (j >= P2) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = tile_rows[t * 16 + 4 * r + kk];
        if (m >= 0) u[static_cast<int64_t>(m) * P2 + j] = static_cast<R>(acc[ch][r]);
      }
    }
  }
}

void launch_tile_fill(const int32_t* tile_rows, int64_t nslots, const int64_t* rowptr, const int32_t* col,
                      const double* val, const int64_t* coff, const int32_t* cols, const int64_t* voff, double* tv,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_tile_fill, dim3(static_cast<unsigned>((nslots + 255) / 256)), dim3(256), 0, st, tile_rows,
                     nslots, rowptr, col, val, coff, cols, voff, tv);
}

template <typename R>
void launch_corr_tile(const int32_t* tile_rows, int64_t ntiles, const int64_t* coff, const int32_t* cols,
                      const int64_t* voff, const double* tv, const void* x, int P, void* u, hipStream_t st) {
  hipLaunchKernelGGL((k_corr_tile<R>), dim3(static_cast<unsigned>((ntiles + kTileWaves - 1) / kTileWaves)),
                     dim3(64 * kTileWaves), 0, st, tile_rows, ntiles, coff, cols, voff, tv,
                     static_cast<const R*>(x), 2 * P, static_cast<R*>(u));
}

template void launch_corr_tile<double>(const int32_t*, int64_t, const int64_t*, const int32_t*, const int64_t*,
                                       const double*, const void*, int, void*, hipStream_t);
template void launch_corr_tile<float>(const int32_t*, int64_t, const int64_t*, const int32_t*, const int64_t*,
                                      const double*, const void*, int, void*, hipStream_t);

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

int launch_corr_count(const CorrArgs& a, const int32_t* s3, const int32_t* box_start, int64_t* rowcount,
                      hipStream_t st) {
  unsigned nb = static_cast<unsigned>((a.N + 255) / 256);
  hipLaunchKernelGGL(k_corr_count, dim3(nb), dim3(256), 0, st, a, s3, box_start, rowcount);
  return FFTPIM_OK;
}

template <int Q>
static void fill_q(bool cplx_vals, bool adj, const CorrArgs& a, const int32_t* s3, const double* u3,
                   const double* pos3, const double* u3c, const double* pos3c, const int32_t* box_start,
                   const void* g0tab, const int64_t* rowptr, int32_t* col, void* val, void* val_adj, hipStream_t st) {
  // one wavefront per row (kFillRPW rows each), the table in LDS beside
  // the wave lists when both fit, else read from global memory
  const size_t tab = tab_lds_bytes(a.W, cplx_vals);
  const bool lt = tab + fill_list_bytes() <= kTabLdsBytes;
  const size_t lds = (lt ? tab : 0) + fill_list_bytes();
  const int64_t per_block = static_cast<int64_t>(kFillWaves) * kFillRPW;
  const unsigned nb = static_cast<unsigned>((a.N + per_block - 1) / per_block);
  const cplx<double>* g = static_cast<const cplx<double>*>(g0tab);
#define FFTPIM_FILL(C, J)                                                                                     \
  do {                                                                                                        \
    if (lt)                                                                                                   \
      hipLaunchKernelGGL((k_corr_fill_wave<Q, C, J, true>), dim3(nb), dim3(64 * kFillWaves), lds, st, a, s3,  \
                         u3, pos3, u3c, pos3c, box_start, g, rowptr, col, val, val_adj);                      \
    else                                                                                                      \
      hipLaunchKernelGGL((k_corr_fill_wave<Q, C, J, false>), dim3(nb), dim3(64 * kFillWaves), lds, st, a, s3, \
                         u3, pos3, u3c, pos3c, box_start, g, rowptr, col, val, val_adj);                      \
  } while (0)
  if (!cplx_vals)
    FFTPIM_FILL(false, false);
  else if (adj)
    FFTPIM_FILL(true, true);
  else
    FFTPIM_FILL(true, false);
#undef FFTPIM_FILL
}

int launch_corr_fill(int q, bool cplx_vals, bool adj, const CorrArgs& a, const int32_t* s3, const double* u3,
                     const double* pos3, const double* u3c, const double* pos3c, const int32_t* box_start,
                     const void* g0tab, const int64_t* rowptr, int32_t* col, void* val, void* val_adj,
                     hipStream_t st) {
  switch (q) {
    case 1: fill_q<1>(cplx_vals, adj, a, s3, u3, pos3, u3c, pos3c, box_start, g0tab, rowptr, col, val, val_adj, st); break;
    case 2: fill_q<2>(cplx_vals, adj, a, s3, u3, pos3, u3c, pos3c, box_start, g0tab, rowptr, col, val, val_adj, st); break;
    case 3: fill_q<3>(cplx_vals, adj, a, s3, u3, pos3, u3c, pos3c, box_start, g0tab, rowptr, col, val, val_adj, st); break;
    case 4: fill_q<4>(cplx_vals, adj, a, s3, u3, pos3, u3c, pos3c, box_start, g0tab, rowptr, col, val, val_adj, st); break;
    case 5: fill_q<5>(cplx_vals, adj, a, s3, u3, pos3, u3c, pos3c, box_start, g0tab, rowptr, col, val, val_adj, st); break;
    case 6: fill_q<6>(cplx_vals, adj, a, s3, u3, pos3, u3c, pos3c, box_start, g0tab, rowptr, col, val, val_adj, st); break;
    case 7: fill_q<7>(cplx_vals, adj, a, s3, u3, pos3, u3c, pos3c, box_start, g0tab, rowptr, col, val, val_adj, st); break;
    case 8: fill_q<8>(cplx_vals, adj, a, s3, u3, pos3, u3c, pos3c, box_start, g0tab, rowptr, col, val, val_adj, st); break;
    default: return FFTPIM_ERR_UNSUPPORTED;
  }
  return FFTPIM_OK;
}

template <typename R>
void launch_corr_spmv(bool cplx_vals, const int64_t* rowptr, const int32_t* col, const void* val, int64_t N,
                      const int32_t* order, int64_t nslots, const void* qint, int P, void* uint, bool accumulate,
                      hipStream_t st) {
  const int acc = accumulate ? 1 : 0;
  const cplx<R>* q = static_cast<const cplx<R>*>(qint);
  cplx<R>* u = static_cast<cplx<R>*>(uint);
  const unsigned nb = static_cast<unsigned>(((order != nullptr ? nslots : N) + 3) / 4);
  if (P > 4) {
#define FFTPIM_SPMM(LPV)                                                                                   \
  do {                                                                                                     \
    if (cplx_vals)                                                                                         \
      hipLaunchKernelGGL((k_corr_spmm<R, true, LPV>), dim3(nb), dim3(256), 0, st, rowptr, col, val, N, order, q, P, u, acc); \
    else                                                                                                   \
      hipLaunchKernelGGL((k_corr_spmm<R, false, LPV>), dim3(nb), dim3(256), 0, st, rowptr, col, val, N, order, q, P, u, acc); \
  } while (0)
    if (P <= 8)
      FFTPIM_SPMM(8);
    else if (P <= 16)
      FFTPIM_SPMM(16);
    else if (P <= 32)
      FFTPIM_SPMM(32);
    else
      FFTPIM_SPMM(64);
#undef FFTPIM_SPMM
    return;
  }
#define FFTPIM_SPMV(PBV)                                                                                   \
  do {                                                                                                     \
    dim3 gr(nb, (P + PBV - 1) / PBV);                                                                      \
    if (cplx_vals)                                                                                         \
      hipLaunchKernelGGL((k_corr_spmv<R, true, PBV>), gr, dim3(256), 0, st, rowptr, col, val, N, order, q, P, u, acc); \
    else                                                                                                   \
      hipLaunchKernelGGL((k_corr_spmv<R, false, PBV>), gr, dim3(256), 0, st, rowptr, col, val, N, order, q, P, u, acc); \
  } while (0)
  if (P >= 8)
    FFTPIM_SPMV(8);
  else if (P >= 4)
    FFTPIM_SPMV(4);
  else if (P >= 2)
    FFTPIM_SPMV(2);
  else
    FFTPIM_SPMV(1);
#undef FFTPIM_SPMV
}

template void launch_corr_spmv<double>(bool, const int64_t*, const int32_t*, const void*, int64_t, const int32_t*,
                                       int64_t, const void*, int, void*, bool, hipStream_t);
template void launch_corr_spmv<float>(bool, const int64_t*, const int32_t*, const void*, int64_t, const int32_t*,
                                      int64_t, const void*, int, void*, bool, hipStream_t);

}  // namespace fftpim
