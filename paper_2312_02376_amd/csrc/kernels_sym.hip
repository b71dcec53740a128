// Near-zone correction (Sec. 3.3 Step 4, Eq. (er)) for in-cell pairs, stored
// once per unordered pair of near-grid boxes.
//
// For image 0 the entry X_0(m, n) = G0(r_m - r_n) - G_grid,0(m, n) is symmetric
// in (m, n) (both terms are even in r_m - r_n and the double sum of Eq. (er_2)
// is symmetric), so the block of box pair (B, B') with B <= B' serves both
// u_B += X x_B' and u_B' += X^T x_B.  The conjugate transpose of this part is
// conj(X conj(v)), so the same values serve the adjoint.  Close images (i != 0)
// are not symmetric under a phase shift and stay in a separate CSR.
//
// Apply: one wavefront per work item (a box and a run of its lane groups)
// reads every block once, lanes over the blocks' columns: the column sums
// X^T x_B (for the partner box) accumulate in registers, the row sums X x_B'
// come from a register reduce-scatter across the wavefront.  Row sums go to
// per-item partials, column sums to per-group partials; a second kernel adds,
// for every box, its items' partials and the column partials addressed to
// it, in a fixed order (no atomics).
#include "kernels.h"

namespace fftpim {

// ---------------------------------------------------------------------------
// plan time: block values
// ---------------------------------------------------------------------------

template <int Q, bool CPLX>
__global__ void __launch_bounds__(64) k_sym_fill(SymArgs a, const double* __restrict__ w3,
                                                 const double* __restrict__ pos3, const cplx<double>* __restrict__ g0tab,
                                                 void* __restrict__ vals) {
  constexpr int D = 2 * Q + 1;
  __shared__ double gr[D * D * D], gi[D * D * D];
  const int64_t pr = blockIdx.x;
  const int kb = a.pair_ebox_o[pr], kbp = a.pair_ebox_s[pr];
  const int B = a.ebox[kb], Bp = a.ebox[kbp];
  const int bz = B % a.nb[2], by = (B / a.nb[2]) % a.nb[1], bx = B / (a.nb[2] * a.nb[1]);
  const int cz = Bp % a.nb[2], cy = (Bp / a.nb[2]) % a.nb[1], cx = Bp / (a.nb[2] * a.nb[1]);
  const int Dl[3] = {bx - cx, by - cy, bz - cz};
  // the block's slice of the G0 node table: offsets Delta + d, d in [-q, q]^3
  for (int t = threadIdx.x; t < D * D * D; t += blockDim.x) {
    const int dz = t % D - Q, dy = (t / D) % D - Q, dx = t / (D * D) - Q;
    const int64_t k = (static_cast<int64_t>(Dl[0] + dx + a.R) * a.W + (Dl[1] + dy + a.R)) * a.W + (Dl[2] + dz + a.R);
    gr[t] = g0tab[k].x;
    gi[t] = g0tab[k].y;
  }
  __syncthreads();
  const int m0 = a.box_start[B], nB = a.box_start[B + 1] - m0;
  const int n0 = a.box_start[Bp], nBp = a.box_start[Bp + 1] - n0;
  const int64_t voff = a.pair_voff[pr];
  const int64_t stride = a.pair_stride[pr];
  const int64_t N = a.N;
  for (int e = threadIdx.x; e < nB * nBp; e += blockDim.x) {
    const int r = e / nBp, c = e - r * nBp;
    const int m = m0 + r, n = n0 + c;
    double C[3][D];
    for (int ax = 0; ax < 3; ++ax) {
      double wm[Q + 1], wn[Q + 1];
      for (int k = 0; k <= Q; ++k) {
        wm[k] = w3[(ax * (Q + 1) + k) * N + m];
        wn[k] = w3[(ax * (Q + 1) + k) * N + n];
      }
      for (int d = -Q; d <= Q; ++d) {
        double s = 0.0;
        for (int aa = max(0, d); aa <= min(Q, Q + d); ++aa) s += wm[aa] * wn[aa - d];
        C[ax][d + Q] = s;
      }
    }
    double sr = 0.0, si = 0.0;
    for (int dx = 0; dx < D; ++dx)
      for (int dy = 0; dy < D; ++dy) {
        const double cxy = C[0][dx] * C[1][dy];
        const int t0 = (dx * D + dy) * D;
        double zr = 0.0, zi = 0.0;
        for (int dz = 0; dz < D; ++dz) {
          zr += C[2][dz] * gr[t0 + dz];
          if (CPLX) zi += C[2][dz] * gi[t0 + dz];
        }
        sr += cxy * zr;
        si += cxy * zi;
      }
    double er = 0.0, ei = 0.0;
    if (m != n) {
      const double dx = pos3[m] - pos3[n], dy = pos3[N + m] - pos3[N + n], dz = pos3[2 * N + m] - pos3[2 * N + n];
      const double rr = sqrt(dx * dx + dy * dy + dz * dz);
      const double inv = (a.k0_im != 0.0 ? exp(a.k0_im * rr) : 1.0) / (4.0 * M_PI * rr);
      if (CPLX) {
        double s, c2;
        sincos(a.k0 * rr, &s, &c2);
        er = c2 * inv;
        ei = -s * inv;
      } else {
        er = inv;
      }
    }
    const int64_t idx = voff + static_cast<int64_t>(r) * stride + c;
    if (CPLX)
      static_cast<cplx<double>*>(vals)[idx] = cmake<double>(er - sr, ei - si);
    else
      static_cast<double*>(vals)[idx] = er - sr;
  }
}

// ---------------------------------------------------------------------------
// apply
// ---------------------------------------------------------------------------

typedef double dbl2v __attribute__((ext_vector_type(2)));

// Inputs and outputs of one apply: planes [0, P1) come from x1 (stride P1) and
// go to u1, planes [P1, P) from x2 / to u2 (stride P - P1), each set with its
// own conjugation (a forward and a conjugate-transpose apply can share one
// pass over the stored blocks: conj(X conj(v)) is the transpose apply).
template <typename R>
struct SymIO {
  const cplx<R>* x1;
  const cplx<R>* x2;
  cplx<R>* u1;
  cplx<R>* u2;
  int P1, P;
  int conj1, conj2;
};

template <typename R>
__device__ inline void load_planes(const SymIO<R>& io, int64_t pt, int p, double& re, double& im) {
  const bool first = p < io.P1;
  const cplx<R> v = first ? io.x1[pt * io.P1 + p] : io.x2[pt * (io.P - io.P1) + (p - io.P1)];
  re = static_cast<double>(v.x);
  im = (first ? io.conj1 : io.conj2) ? -static_cast<double>(v.y) : static_cast<double>(v.y);
}

// Reduce-scatter of 8 values per lane over the 64 lanes of a wavefront:
// afterwards lanes with bits 5,4,3 = (b5, b4, b3) hold the total of value
// 4 b5 + 2 b4 + b3 (all lanes of an 8-lane group hold the same total).
__device__ inline double wave_reduce_scatter8(double v[8], int lane) {
  const bool u32 = (lane & 32) != 0, u16 = (lane & 16) != 0, u8 = (lane & 8) != 0;
  double a[4], b[2];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double send = u32 ? v[k] : v[k + 4];
    const double keep = u32 ? v[k + 4] : v[k];
    a[k] = keep + __shfl_xor(send, 32, 64);
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double send = u16 ? a[k] : a[k + 2];
    const double keep = u16 ? a[k + 2] : a[k];
    b[k] = keep + __shfl_xor(send, 16, 64);
  }
  double s = (u8 ? b[1] : b[0]) + __shfl_xor(u8 ? b[0] : b[1], 8, 64);
  s += __shfl_xor(s, 4, 64);
  s += __shfl_xor(s, 2, 64);
  s += __shfl_xor(s, 1, 64);
  return s;
}

// One wavefront per work item (a box B and a run of its lane groups).  A lane
// owns one column of the group; eight rows of values are loaded back to back,
// each lane accumulates its column sum (X^T x_B, sent to the partner box) in
// registers, and the row sums (X x_B' over the group's pairs) come from a
// register reduce-scatter.  The group record alone gives every address, so
// the value and source loads of a group issue without waiting on other
// tables.  LDS holds x_B and the row accumulators.
template <typename R, bool CPLX, int PP>
__device__ inline void sym_rows(const double* __restrict__ vr, const cplx<double>* __restrict__ vc,
                                const cplx<double>* xb, cplx<double>* yacc, int nB, int P, int pg, int lane, bool act,
                                int64_t voff, int64_t stride, const double (&xsr)[PP], const double (&xsi)[PP],
                                double (&zr)[PP], double (&zi)[PP]) {
  const int krow = ((lane >> 5) & 1) * 4 + ((lane >> 4) & 1) * 2 + ((lane >> 3) & 1);
  for (int r0 = 0; r0 < nB; r0 += 8) {
    double wr[8], wi[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      wr[k] = 0.0;
      wi[k] = 0.0;
      if (act && r0 + k < nB) {
        const int64_t idx = voff + static_cast<int64_t>(r0 + k) * stride + lane;
        // the values are streamed once per apply: nontemporal loads keep
        // them from displacing reused data in the caches
        if (CPLX) {
          wr[k] = __builtin_nontemporal_load(reinterpret_cast<const double*>(vc + idx));
          wi[k] = __builtin_nontemporal_load(reinterpret_cast<const double*>(vc + idx) + 1);
        } else {
          wr[k] = __builtin_nontemporal_load(vr + idx);
        }
      }
    }
    // every plane of the group uses the rows just loaded
#pragma unroll
    for (int pp = 0; pp < PP; ++pp) {
      const int p = pg + pp;
      if (p >= P) break;
      double pr_[8], pi_[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (r0 + k < nB) {
          const cplx<double> xv = xb[(r0 + k) * P + p];
          zr[pp] += wr[k] * xv.x - wi[k] * xv.y;
          zi[pp] += wr[k] * xv.y + wi[k] * xv.x;
        }
        pr_[k] = wr[k] * xsr[pp] - wi[k] * xsi[pp];
        pi_[k] = wr[k] * xsi[pp] + wi[k] * xsr[pp];
      }
      const double sr = wave_reduce_scatter8(pr_, lane);
      const double si = wave_reduce_scatter8(pi_, lane);
      if ((lane & 7) == 0 && r0 + krow < nB) {
        cplx<double> acc = yacc[(r0 + krow) * P + p];
        acc.x += sr;
        acc.y += si;
        yacc[(r0 + krow) * P + p] = acc;
      }
    }
  }
}

// PP planes are processed per pass over a group's values (all planes when
// P <= PP, so forward and transpose applies fused into one call read every
// block once).
template <typename R, bool CPLX, int PP>
__global__ void __launch_bounds__(64) k_sym_apply(SymArgs a, const SymGroup* __restrict__ groups,
                                                  const void* __restrict__ vals, SymIO<R> io,
                                                  cplx<double>* __restrict__ ypart, cplx<double>* __restrict__ zpart) {
  extern __shared__ unsigned char lds_raw[];
  const int P = io.P;
  const int item = a.item_order[blockIdx.x];
  const int lane = threadIdx.x;
  const int B = a.ebox[a.item_ebox[item]];
  const int m0 = a.box_start[B], nB = a.box_start[B + 1] - m0;
  cplx<double>* xb = reinterpret_cast<cplx<double>*>(lds_raw);          // [nB][P]
  cplx<double>* yacc = xb + static_cast<int64_t>(a.max_box) * P;         // [nB][P]
  for (int t = lane; t < nB * P; t += 64) {
    double re, im;
    load_planes<R>(io, m0 + t / P, t % P, re, im);
    xb[t] = cmake<double>(re, im);
    yacc[t] = cmake<double>(0.0, 0.0);
  }
  __syncthreads();
  const double* vr = static_cast<const double*>(vals);
  const cplx<double>* vc = static_cast<const cplx<double>*>(vals);
  const int64_t gend = a.item_gbeg[item + 1];
  for (int64_t gi = a.item_gbeg[item]; gi < gend; ++gi) {
    // the record alone gives every address of the group (read through the
    // scalar cache: the table is read-only here)
    const SymGroup g = groups[gi];
    const bool act = lane < g.cum;
    // source point of this lane's column
    int n = g.n0[0] + lane;
    if (lane >= g.end[0]) n = g.n0[1] + lane - g.end[0];
    if (lane >= g.end[1]) n = g.n0[2] + lane - g.end[1];
    if (lane >= g.end[2]) n = g.n0[3] + lane - g.end[2];
    const bool wr = lane < (g.cum + kSymZAlign - 1) / kSymZAlign * kSymZAlign;
    for (int pg = 0; pg < P; pg += PP) {
      double xsr[PP], xsi[PP], zr[PP], zi[PP];
#pragma unroll
      for (int pp = 0; pp < PP; ++pp) {
        xsr[pp] = xsi[pp] = zr[pp] = zi[pp] = 0.0;
        if (act && pg + pp < P) load_planes<R>(io, n, pg + pp, xsr[pp], xsi[pp]);
      }
      sym_rows<R, CPLX, PP>(vr, vc, xb, yacc, nB, P, pg, lane, act, g.voff, g.stride, xsr, xsi, zr, zi);
      // the run is written whole, padded to 64-byte segments (padding and
      // diagonal-block columns are never read)
      if (wr) {
#pragma unroll
        for (int pp = 0; pp < PP; ++pp)
          if (pg + pp < P) zpart[(g.zoff + lane) * P + pg + pp] = cmake<double>(zr[pp], zi[pp]);
      }
    }
  }
  __syncthreads();
  const int64_t yoff = a.item_yoff[item];
  for (int t = lane; t < nB * P; t += 64) ypart[yoff * P + t] = yacc[t];
}

// One workgroup per non-empty box B.  Its partial sums come in runs of n_B P
// contiguous values: one run per work item of B (row sums, ypart) and one
// per box sending column sums to B (zpart, senders in box order).  Threads
// split into S slices of n_B P lanes; slice s adds runs s, s + S, ...; the
// slices are then added in slice order (a fixed order: results do not depend
// on scheduling).
constexpr int kGatherThreads = 256;

template <typename R>
__global__ void __launch_bounds__(kGatherThreads) k_sym_gather(SymArgs a, const cplx<double>* __restrict__ ypart,
                                                               const cplx<double>* __restrict__ zpart, SymIO<R> io,
                                                               int accumulate) {
  __shared__ double sr_[kGatherThreads], si_[kGatherThreads];
  const int P = io.P;
  const int kb = blockIdx.x;
  const int t = threadIdx.x;
  const int B = a.ebox[kb];
  const int m0 = a.box_start[B], nB = a.box_start[B + 1] - m0;
  const int it0 = a.ebox_item_beg[kb], nit = a.ebox_item_beg[kb + 1] - it0;
  const int64_t y0 = a.item_yoff[it0] * P;
  const int64_t ip0 = a.in_ptr[kb];
  const int run = nB * P;
  const int64_t nruns = nit + (a.in_ptr[kb + 1] - ip0);
  const int S = run <= kGatherThreads ? kGatherThreads / run : 1;
  for (int e0 = 0; e0 < run; e0 += kGatherThreads) {
    const int s = S > 1 ? t / run : 0;
    const int e = S > 1 ? t - s * run : e0 + t;
    const bool act = s < S && e < run;
    double xr = 0.0, xi = 0.0;
    if (act) {
      // runs s, s + S, ... in increasing order: the row partials of the
      // box's items, then the column partials; loads are issued kU at a time
      // (the column runs through their index first) so their latencies
      // overlap
      constexpr int kU = 8;
      int64_t k = s;
      for (; k + (kU - 1) * S < nit; k += kU * S) {
        cplx<double> v[kU];
#pragma unroll
        for (int j = 0; j < kU; ++j) v[j] = ypart[y0 + (k + j * S) * run + e];
#pragma unroll
        for (int j = 0; j < kU; ++j) {
          xr += v[j].x;
          xi += v[j].y;
        }
      }
      for (; k < nit; k += S) {
        const cplx<double> v = ypart[y0 + k * run + e];
        xr += v.x;
        xi += v.y;
      }
      for (; k + (kU - 1) * S < nruns; k += kU * S) {
        int64_t zb[kU];
#pragma unroll
        for (int j = 0; j < kU; ++j) zb[j] = a.in_base[ip0 + k + j * S - nit];
        cplx<double> v[kU];
#pragma unroll
        for (int j = 0; j < kU; ++j) v[j] = zpart[zb[j] * P + e];
#pragma unroll
        for (int j = 0; j < kU; ++j) {
          xr += v[j].x;
          xi += v[j].y;
        }
      }
      for (; k < nruns; k += S) {
        const cplx<double> v = zpart[a.in_base[ip0 + k - nit] * P + e];
        xr += v.x;
        xi += v.y;
      }
    }
    sr_[t] = xr;
    si_[t] = xi;
    __syncthreads();
    const int nout = S > 1 ? run : min(kGatherThreads, run - e0);
    if (t < nout) {
      double tr = 0.0, ti = 0.0;
      for (int k = 0; k < S; ++k) {
        tr += sr_[k * (S > 1 ? run : 0) + t];
        ti += si_[k * (S > 1 ? run : 0) + t];
      }
      const int e = S > 1 ? t : e0 + t;  // (point, plane) slot within the box
      const int r = e / P, p = e - (e / P) * P;
      const bool first = p < io.P1;
      if (first ? io.conj1 : io.conj2) ti = -ti;
      cplx<R>* o = first ? io.u1 + static_cast<int64_t>(m0 + r) * io.P1 + p
                         : io.u2 + static_cast<int64_t>(m0 + r) * (P - io.P1) + (p - io.P1);
      cplx<R> out = cmake<R>(static_cast<R>(tr), static_cast<R>(ti));
      if (accumulate) out = cadd(*o, out);
      *o = out;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

int launch_sym_fill(int q, bool cplx_vals, const SymArgs& a, const double* w3, const double* pos3,
                    const void* g0tab, void* vals, hipStream_t st) {
  const cplx<double>* g = static_cast<const cplx<double>*>(g0tab);
#define FFTPIM_SYMFILL(QV)                                                                                  \
  do {                                                                                                      \
    if (cplx_vals)                                                                                          \
      hipLaunchKernelGGL((k_sym_fill<QV, true>), dim3(static_cast<unsigned>(a.npairs)), dim3(64), 0, st, a, w3, \
                         pos3, g, vals);                                                                    \
    else                                                                                                    \
      hipLaunchKernelGGL((k_sym_fill<QV, false>), dim3(static_cast<unsigned>(a.npairs)), dim3(64), 0, st, a, \
                         w3, pos3, g, vals);                                                                \
  } while (0)
  switch (q) {
    case 1: FFTPIM_SYMFILL(1); break;
    case 2: FFTPIM_SYMFILL(2); break;
    case 3: FFTPIM_SYMFILL(3); break;
    case 4: FFTPIM_SYMFILL(4); break;
    case 5: FFTPIM_SYMFILL(5); break;
    case 6: FFTPIM_SYMFILL(6); break;
    case 7: FFTPIM_SYMFILL(7); break;
    case 8: FFTPIM_SYMFILL(8); break;
    default: return FFTPIM_ERR_UNSUPPORTED;
  }
#undef FFTPIM_SYMFILL
  return FFTPIM_OK;
}

template <typename R>
void launch_sym_apply(bool cplx_vals, const SymArgs& a, const void* vals, const void* x1, const void* x2, int P1,
                      int P, bool conj1, bool conj2, void* ypart, void* zpart, void* u1, void* u2, bool accumulate,
                      hipStream_t st) {
  const size_t lds = static_cast<size_t>(2) * a.max_box * P * sizeof(cplx<double>);
  SymIO<R> io;
  io.x1 = static_cast<const cplx<R>*>(x1);
  io.x2 = static_cast<const cplx<R>*>(x2);
  io.u1 = static_cast<cplx<R>*>(u1);
  io.u2 = static_cast<cplx<R>*>(u2);
  io.P1 = P1;
  io.P = P;
  io.conj1 = conj1 ? 1 : 0;
  io.conj2 = conj2 ? 1 : 0;
  cplx<double>* yp = static_cast<cplx<double>*>(ypart);
  cplx<double>* zp = static_cast<cplx<double>*>(zpart);
  const dim3 gr(static_cast<unsigned>(a.nitems));
#define FFTPIM_SYMAPPLY(C, PPV) \
  hipLaunchKernelGGL((k_sym_apply<R, C, PPV>), gr, dim3(64), lds, st, a, a.groups, vals, io, yp, zp)
  if (cplx_vals) {
    if (P == 1) FFTPIM_SYMAPPLY(true, 1); else if (P == 2) FFTPIM_SYMAPPLY(true, 2); else FFTPIM_SYMAPPLY(true, 4);
  } else {
    if (P == 1) FFTPIM_SYMAPPLY(false, 1); else if (P == 2) FFTPIM_SYMAPPLY(false, 2); else FFTPIM_SYMAPPLY(false, 4);
  }
#undef FFTPIM_SYMAPPLY
  hipLaunchKernelGGL((k_sym_gather<R>), dim3(static_cast<unsigned>(a.nebox)), dim3(kGatherThreads), 0, st, a, yp, zp, io,
                     accumulate ? 1 : 0);
}

template void launch_sym_apply<double>(bool, const SymArgs&, const void*, const void*, const void*, int, int, bool,
                                       bool, void*, void*, void*, void*, bool, hipStream_t);
template void launch_sym_apply<float>(bool, const SymArgs&, const void*, const void*, const void*, int, int, bool,
                                      bool, void*, void*, void*, void*, bool, hipStream_t);

}  // namespace fftpim
