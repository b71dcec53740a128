// Near-zone grid kernels (Sec. 3.3, Steps 1-3) and shared helpers:
//   * pack / unpack between the caller's [nrhs][N] arrays and the plan-order,
//     point-major complex "planes" used inside (two real right-hand sides
//     share one complex plane when the kernel is real);
//   * projection onto the near grid (Step 1) as an atomic-free gather: every
//     grid node sums the contributions of the points in the (q+1)^3 boxes
//     whose stencils cover it;
//   * zero-padded FFT passes (Step 2) with radix-2 transforms in LDS; the
//     x-axis pass fuses forward transform, multiplication by the kernel
//     spectrum and inverse transform;
//   * interpolation back to the points (Step 3);
//   * the near-zone kernel table G^p_near at grid offsets (plan time).
#include "kernels.h"

namespace fftpim {

// ---------------------------------------------------------------------------
// pack / unpack
// ---------------------------------------------------------------------------

template <typename R, bool REAL_IN>
__global__ void k_pack(const void* __restrict__ qu, cplx<R>* __restrict__ qint,
                       const int32_t* __restrict__ perm, int64_t N, int nrhs, int P, int use_perm) {
  int64_t tid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (tid >= N * P) return;
  int p = static_cast<int>(tid / N);
  int64_t m = tid - static_cast<int64_t>(p) * N;
  int64_t src = use_perm ? perm[m] : m;
  cplx<R> v;
  if (REAL_IN) {
    const R* q = static_cast<const R*>(qu);
    int r0 = 2 * p, r1 = 2 * p + 1;
    v.x = r0 < nrhs ? q[static_cast<int64_t>(r0) * N + src] : R(0);
    v.y = r1 < nrhs ? q[static_cast<int64_t>(r1) * N + src] : R(0);
  } else {
    const cplx<R>* q = static_cast<const cplx<R>*>(qu);
    v = q[static_cast<int64_t>(p) * N + src];
  }
  qint[m * P + p] = v;
}

// Sums the parts of the apply that were computed (near grid, correction, far
// zone; absent parts are null) in that fixed order and writes the caller's
// layout, removing a per-plane mean when one is given.
template <typename R, bool REAL_OUT>
__global__ void k_unpack(PartPtrs<R> parts, void* __restrict__ uu, const int32_t* __restrict__ perm, int64_t N,
                         int nrhs, int P, int use_perm, const double* __restrict__ mean) {
  int64_t tid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (tid >= N * P) return;
  int p = static_cast<int>(tid / N);
  int64_t m = tid - static_cast<int64_t>(p) * N;
  int64_t dst = use_perm ? perm[m] : m;
  cplx<R> v = parts.sum(m * P + p);
  if (mean) {
    v.x -= static_cast<R>(mean[2 * p]);
    v.y -= static_cast<R>(mean[2 * p + 1]);
  }
  if (REAL_OUT) {
    R* u = static_cast<R*>(uu);
    int r0 = 2 * p, r1 = 2 * p + 1;
    if (r0 < nrhs) u[static_cast<int64_t>(r0) * N + dst] = v.x;
    if (r1 < nrhs) u[static_cast<int64_t>(r1) * N + dst] = v.y;
  } else {
    cplx<R>* u = static_cast<cplx<R>*>(uu);
    u[static_cast<int64_t>(p) * N + dst] = v;
  }
}

// Tiled forms of pack / unpack for several planes: a block transposes 64
// points x 32 planes through LDS, so both the caller's [rhs][N] side and the
// point-major [N][P] side are read and written in contiguous runs.
constexpr int kTpPts = 64, kTpPl = 32;

template <typename R, bool REAL_IN>
__global__ void __launch_bounds__(256) k_pack_tiled(const void* __restrict__ qu, cplx<R>* __restrict__ qint,
                                                    const int32_t* __restrict__ perm, int64_t N, int nrhs, int P,
                                                    int use_perm) {
  __shared__ cplx<R> tile[kTpPl][kTpPts + 1];
  const int64_t m0 = static_cast<int64_t>(blockIdx.x) * kTpPts;
  const int pc = blockIdx.y * kTpPl;
  const int t = threadIdx.x;
  for (int i = t; i < kTpPl * kTpPts; i += blockDim.x) {
    const int pp = i / kTpPts, mm = i % kTpPts;
    const int64_t m = m0 + mm;
    const int p = pc + pp;
    cplx<R> v = cmake<R>(R(0), R(0));
    if (m < N && p < P) {
      const int64_t src = use_perm ? perm[m] : m;
      if (REAL_IN) {
        const R* q = static_cast<const R*>(qu);
        const int r0 = 2 * p, r1 = 2 * p + 1;
        v.x = r0 < nrhs ? q[static_cast<int64_t>(r0) * N + src] : R(0);
        v.y = r1 < nrhs ? q[static_cast<int64_t>(r1) * N + src] : R(0);
      } else {
        v = static_cast<const cplx<R>*>(qu)[static_cast<int64_t>(p) * N + src];
      }
    }
    tile[pp][mm] = v;
  }
  __syncthreads();
  for (int i = t; i < kTpPl * kTpPts; i += blockDim.x) {
    const int mm = i / kTpPl, pp = i % kTpPl;
    const int64_t m = m0 + mm;
    const int p = pc + pp;
    if (m < N && p < P) qint[m * P + p] = tile[pp][mm];
  }
}

template <typename R, bool REAL_OUT>
__global__ void __launch_bounds__(256) k_unpack_tiled(PartPtrs<R> parts, void* __restrict__ uu,
                                                      const int32_t* __restrict__ perm, int64_t N, int nrhs, int P,
                                                      int use_perm, const double* __restrict__ mean) {
  __shared__ cplx<R> tile[kTpPl][kTpPts + 1];
  const int64_t m0 = static_cast<int64_t>(blockIdx.x) * kTpPts;
  const int pc = blockIdx.y * kTpPl;
  const int t = threadIdx.x;
  for (int i = t; i < kTpPl * kTpPts; i += blockDim.x) {
    const int mm = i / kTpPl, pp = i % kTpPl;
    const int64_t m = m0 + mm;
    const int p = pc + pp;
    if (m < N && p < P) {
      cplx<R> v = parts.sum(m * P + p);
      if (mean) {
        v.x -= static_cast<R>(mean[2 * p]);
        v.y -= static_cast<R>(mean[2 * p + 1]);
      }
      tile[pp][mm] = v;
    }
  }
  __syncthreads();
  for (int i = t; i < kTpPl * kTpPts; i += blockDim.x) {
    const int pp = i / kTpPts, mm = i % kTpPts;
    const int64_t m = m0 + mm;
    const int p = pc + pp;
    if (m >= N || p >= P) continue;
    const int64_t dst = use_perm ? perm[m] : m;
    const cplx<R> v = tile[pp][mm];
    if (REAL_OUT) {
      R* u = static_cast<R*>(uu);
      const int r0 = 2 * p, r1 = 2 * p + 1;
      if (r0 < nrhs) u[static_cast<int64_t>(r0) * N + dst] = v.x;
      if (r1 < nrhs) u[static_cast<int64_t>(r1) * N + dst] = v.y;
    } else {
      static_cast<cplx<R>*>(uu)[static_cast<int64_t>(p) * N + dst] = v;
    }
  }
}

// Per-plane sums over points, deterministic, in two stages:
// out[4p + 0/1] = sum of re/im, out[4p + 2/3] = sum of |re| / |im|.
// Stage 1: block (chunk c, plane tile) sums kPlaneSumChunk points; its 256
// threads are 4 rows of 64 planes (coalesced across planes) and the rows are
// added in order.  Stage 2: one thread per plane adds the chunks in order.
constexpr int kPlaneSumChunk = 1024;

template <typename R>
__global__ void __launch_bounds__(256) k_plane_sums_part(PartPtrs<R> v, int64_t N, int P, double* __restrict__ part) {
  __shared__ double sh[4][4][64];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int p = blockIdx.y * 64 + tx;
  const int64_t m0 = static_cast<int64_t>(blockIdx.x) * kPlaneSumChunk;
  const int64_t m1 = min<int64_t>(N, m0 + kPlaneSumChunk);
  double a = 0, b = 0, c = 0, d = 0;
  if (p < P) {
    for (int64_t m = m0 + ty; m < m1; m += 4) {
      const cplx<R> t = v.sum(m * P + p);
      a += t.x;
      b += t.y;
      c += fabs(static_cast<double>(t.x));
      d += fabs(static_cast<double>(t.y));
    }
  }
  sh[0][ty][tx] = a;
  sh[1][ty][tx] = b;
  sh[2][ty][tx] = c;
  sh[3][ty][tx] = d;
  __syncthreads();
  if (ty == 0 && p < P) {
    double* o = part + (static_cast<int64_t>(blockIdx.x) * P + p) * 4;
    for (int k = 0; k < 4; ++k) o[k] = ((sh[k][0][tx] + sh[k][1][tx]) + sh[k][2][tx]) + sh[k][3][tx];
  }
}

__global__ void k_plane_sums_final(const double* __restrict__ part, int64_t nchunks, int P, double* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double s[4] = {0, 0, 0, 0};
  for (int64_t c = 0; c < nchunks; ++c)
    for (int k = 0; k < 4; ++k) s[k] += part[(c * P + p) * 4 + k];
  for (int k = 0; k < 4; ++k) out[4 * p + k] = s[k];
}

// Neutrality (Eq. (neutral)) per real right-hand side; latches the status.
__global__ void k_check_neutral(const double* __restrict__ sums, int P, double tol, int* status) {
  for (int p = threadIdx.x; p < P; p += blockDim.x) {
    bool bad = fabs(sums[4 * p + 0]) > tol * fmax(sums[4 * p + 2], 1e-300) ||
               fabs(sums[4 * p + 1]) > tol * fmax(sums[4 * p + 3], 1e-300);
    if (bad) atomicCAS(status, 0, static_cast<int>(FFTPIM_ERR_NOT_NEUTRAL));
  }
}

__global__ void k_mean_from_sums(const double* __restrict__ sums, int P, double invN, double* mean) {
  for (int p = threadIdx.x; p < P; p += blockDim.x) {
    mean[2 * p] = sums[4 * p] * invN;
    mean[2 * p + 1] = sums[4 * p + 1] * invN;
  }
}

// ---------------------------------------------------------------------------
// Step 1: projection onto the near grid (gather form)
// ---------------------------------------------------------------------------

// A block owns a tile of TX x TY x TZ grid nodes (one thread per node) and
// gathers every point whose stencil covers the tile: the points of the boxes
// [tile - q, tile] per axis, which form (TX+q)(TY+q) contiguous runs of the
// box-sorted point list.  Points are staged through LDS in chunks together
// with their 1D Lagrange weights and amplitudes; each thread then sums the
// staged points that cover its node, always in the same order (no atomics,
// bitwise reproducible).  Used below 16 planes, where the few multiply-adds
// per point leave the broadcast reads cheaper than per-lane point lists.
constexpr int kSpreadTX = 4, kSpreadTY = 8, kSpreadTZ = 8, kSpreadChunk = 256;

template <typename R, int Q, int PB>
__global__ void __launch_bounds__(256) k_spread_near(
    GridArgs g, const int32_t* __restrict__ box_start, const int32_t* __restrict__ s3,
    const double* __restrict__ w3, int64_t N, const cplx<R>* __restrict__ qint, int P,
    cplx<R>* __restrict__ grid) {
  constexpr int TX = kSpreadTX, TY = kSpreadTY, TZ = kSpreadTZ;
  // staged bytes per point: weights, amplitudes, box; keep the chunk within 48 KB of LDS
  constexpr int kPerPoint = 3 * (Q + 1) * static_cast<int>(sizeof(R)) + PB * 2 * static_cast<int>(sizeof(R)) + 12;
  constexpr int CH = (kSpreadChunk * kPerPoint <= 49152) ? kSpreadChunk
                     : ((kSpreadChunk / 2) * kPerPoint <= 49152 ? kSpreadChunk / 2 : kSpreadChunk / 4);
  static_assert(CH <= TX * TY * TZ, "one staging thread per chunk slot");
  constexpr int NR = (TX + Q) * (TY + Q);
  __shared__ int rstart[NR + 1];
  __shared__ int rbase[NR];
  __shared__ R sw[CH][3][Q + 1];
  __shared__ int sb[CH][3];
  __shared__ cplx<R> sq[CH][PB];
  const int ntx = (g.n[0] + TX - 1) / TX, nty = (g.n[1] + TY - 1) / TY, ntz = (g.n[2] + TZ - 1) / TZ;
  const int tile = blockIdx.x;
  const int tz = tile % ntz, ty = (tile / ntz) % nty, tx = tile / (ntz * nty);
  (void)ntx;
  const int gx0 = tx * TX, gy0 = ty * TY, gz0 = tz * TZ;
  const int tid = threadIdx.x;
  const int gx = gx0 + tid / (TY * TZ), gy = gy0 + (tid / TZ) % TY, gz = gz0 + tid % TZ;
  const bool valid = gx < g.n[0] && gy < g.n[1] && gz < g.n[2];
  const int p0 = blockIdx.y * PB;
  // runs of the influence region
  const int bx0 = max(0, gx0 - Q), bx1 = min(g.nint[0], gx0 + TX - 1);
  const int by0 = max(0, gy0 - Q), by1 = min(g.nint[1], gy0 + TY - 1);
  const int bz0 = max(0, gz0 - Q), bz1 = min(g.nint[2], gz0 + TZ - 1);
  const int nbx = max(0, bx1 - bx0 + 1), nby = max(0, by1 - by0 + 1);
  const int nr = (bz1 >= bz0) ? nbx * nby : 0;
  if (tid < nr) {
    const int ix = tid / nby, iy = tid % nby;
    const int64_t bf = (static_cast<int64_t>(bx0 + ix) * g.nb[1] + (by0 + iy)) * g.nb[2] + bz0;
    const int64_t bl = bf + (bz1 - bz0);
    rbase[tid] = box_start[bf];
    rstart[tid + 1] = box_start[bl + 1] - box_start[bf];
  }
  __syncthreads();
  if (tid == 0) {
    rstart[0] = 0;
    for (int r = 0; r < nr; ++r) rstart[r + 1] += rstart[r];
  }
  __syncthreads();
  const int total = rstart[nr];
  R ax[PB], ay[PB];
#pragma unroll
  for (int pp = 0; pp < PB; ++pp) ax[pp] = ay[pp] = R(0);
  for (int base = 0; base < total; base += CH) {
    __syncthreads();
    const int k = base + tid;
    if (tid < CH && k < total) {
      int lo = 0, hi = nr - 1;  // run r with rstart[r] <= k < rstart[r + 1]
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rstart[mid] <= k) lo = mid; else hi = mid - 1;
      }
      const int64_t j = rbase[lo] + (k - rstart[lo]);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        sb[tid][c] = s3[c * N + j];
#pragma unroll
        for (int a = 0; a <= Q; ++a) sw[tid][c][a] = static_cast<R>(w3[(c * (Q + 1) + a) * N + j]);
      }
#pragma unroll
      for (int pp = 0; pp < PB; ++pp)
        sq[tid][pp] = (p0 + pp < P) ? qint[j * P + p0 + pp] : cmake<R>(R(0), R(0));
    }
    __syncthreads();
    const int cnt = min(CH, total - base);
    if (valid) {
      for (int i = 0; i < cnt; ++i) {
        const unsigned kx = static_cast<unsigned>(gx - sb[i][0]);
        const unsigned ky = static_cast<unsigned>(gy - sb[i][1]);
        const unsigned kz = static_cast<unsigned>(gz - sb[i][2]);
        if (kx > static_cast<unsigned>(Q) || ky > static_cast<unsigned>(Q) || kz > static_cast<unsigned>(Q)) continue;
        const R w = sw[i][0][kx] * sw[i][1][ky] * sw[i][2][kz];
#pragma unroll
        for (int pp = 0; pp < PB; ++pp) {
          ax[pp] += w * sq[i][pp].x;
          ay[pp] += w * sq[i][pp].y;
        }
      }
    }
  }
  if (valid) {
    const int64_t node = (static_cast<int64_t>(gx) * g.n[1] + gy) * g.n[2] + gz;
#pragma unroll
    for (int pp = 0; pp < PB; ++pp)
      if (p0 + pp < P) grid[node * P + p0 + pp] = cmake<R>(ax[pp], ay[pp]);
  }
}

// The same projection for many planes, each thread summing only the points
// that cover its own nodes.  In the gather above every staged point passes
// through all lanes of a wavefront while its stencil covers few of their
// nodes, so most multiply-add slots are idle.  Here a block owns a tile of
// TX x TY x TZ nodes with one wavefront per x layer; a thread owns two
// z-adjacent nodes (gz, gz + 1).  The boxes are walked one x slab at a time:
// the block stages the slab's points of the tile's y/z influence region
// (1D weights, z box, PB amplitude planes) in LDS, and each thread of a
// layer that the slab covers walks only its own runs - the boxes y in
// [gy - Q, gy] and z in [gz - Q, gz + 1] - so its multiply-adds are useful;
// the lanes of a wavefront differ only in how many points they hold.  Every
// node sums its points in a fixed order (slab, run, point): no atomics,
// bitwise reproducible.
constexpr int kOwnTX = 4, kOwnTY = 8, kOwnTZ = 16;

template <typename R>
struct OwnCfg {
  static constexpr int PB = sizeof(R) == 4 ? 16 : 8;    // planes per pass
  static constexpr int CH = sizeof(R) == 4 ? 192 : 160;  // staged points per chunk
};

template <typename R, int Q>
__global__ void __launch_bounds__(256) k_spread_own(
    GridArgs g, const int32_t* __restrict__ box_start, const int32_t* __restrict__ s3,
    const double* __restrict__ w3, int64_t N, const cplx<R>* __restrict__ qint, int P,
    cplx<R>* __restrict__ grid) {
  constexpr int TX = kOwnTX, TY = kOwnTY, TZ = kOwnTZ, PB = OwnCfg<R>::PB, CH = OwnCfg<R>::CH;
  static_assert(TY * (TZ / 2) == 64 && TX * 64 == 256, "one wavefront per x layer of the tile");
  constexpr int NRY = TY + Q, NBZ = TZ + Q;  // y runs and z boxes of a slab's region
  constexpr int QS = PB + 2;                 // padded plane stride of a staged point (LDS banks)
  __shared__ int bs[NRY][NBZ + 1];           // global start of each box of the slab's runs
  __shared__ int rs[NRY + 1];                // slab-local start of each run
  __shared__ R sw[CH][3][Q + 1];
  __shared__ int sbz[CH];
  __shared__ cplx<R> sq[CH][QS];
  const int nty = (g.n[1] + TY - 1) / TY, ntz = (g.n[2] + TZ - 1) / TZ;
  const int tile = blockIdx.x;
  const int tz = tile % ntz, ty = (tile / ntz) % nty, tx = tile / (ntz * nty);
  const int gx0 = tx * TX, gy0 = ty * TY, gz0 = tz * TZ;
  const int tid = threadIdx.x;
  const int gx = gx0 + tid / 64, gy = gy0 + (tid / (TZ / 2)) % TY, gz = gz0 + 2 * (tid % (TZ / 2));
  const bool valid = gx < g.n[0] && gy < g.n[1] && gz < g.n[2];
  const int p0 = blockIdx.y * PB;
  const int by0 = max(0, gy0 - Q), by1 = min(g.nint[1], gy0 + TY - 1);
  const int bz0 = max(0, gz0 - Q), bz1 = min(g.nint[2], gz0 + TZ - 1);
  const int nry = max(0, by1 - by0 + 1), nbz = max(0, bz1 - bz0 + 1);
  // this thread's runs (slab-independent): y boxes [ly0, ly1], z boxes [lz0, lz1)
  const int ly0 = max(by0, gy - Q) - by0, ly1 = valid ? min(by1, gy) - by0 : -1;
  const int lz0 = max(bz0, gz - Q) - bz0, lz1 = max(lz0, min(bz1, gz + 1) - bz0 + 1);
  R a0x[PB], a0y[PB], a1x[PB], a1y[PB];
#pragma unroll
  for (int pp = 0; pp < PB; ++pp) a0x[pp] = a0y[pp] = a1x[pp] = a1y[pp] = R(0);
  const int bxa = max(0, gx0 - Q), bxb = min(g.nint[0], gx0 + TX - 1);
  for (int bx = bxa; bx <= bxb; ++bx) {
    __syncthreads();  // the previous slab's LDS is no longer read
    for (int i = tid; i < nry * (nbz + 1); i += 256) {
      const int iy = i / (nbz + 1), iz = i % (nbz + 1);
      bs[iy][iz] = box_start[(static_cast<int64_t>(bx) * g.nb[1] + by0 + iy) * g.nb[2] + bz0 + iz];
    }
    __syncthreads();
    if (tid == 0) {
      rs[0] = 0;
      for (int iy = 0; iy < nry; ++iy) rs[iy + 1] = rs[iy] + (bs[iy][nbz] - bs[iy][0]);
    }
    __syncthreads();
    const int total = rs[nry];
    const int kx = gx - bx;  // x weight index; the slab covers this layer when 0 <= kx <= Q
    const bool mine = valid && kx >= 0 && kx <= Q;
    for (int c0 = 0; c0 < total; c0 += CH) {
      const int c1 = min(total, c0 + CH);
      if (c0 > 0) __syncthreads();
      for (int k = c0 + tid; k < c1; k += 256) {
        int lo = 0, hi = nry - 1;  // run with rs[lo] <= k < rs[lo + 1]
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (rs[mid] <= k) lo = mid; else hi = mid - 1;
        }
        const int64_t j = bs[lo][0] + (k - rs[lo]);
        const int s = k - c0;
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int a = 0; a <= Q; ++a) sw[s][c][a] = static_cast<R>(w3[(c * (Q + 1) + a) * N + j]);
        sbz[s] = s3[2 * N + j] - bz0;
#pragma unroll
        for (int pp = 0; pp < PB; ++pp)
          sq[s][pp] = (p0 + pp < P) ? qint[j * P + p0 + pp] : cmake<R>(R(0), R(0));
      }
      __syncthreads();
      if (!mine) continue;
      // walk this thread's runs clipped to [c0, c1) as one flat loop, so
      // that a lane with an empty run does not wait for the others
      int iy = ly0, k = 0, e = 0, ky = 0;
      for (;;) {
        while (k >= e && iy <= ly1) {
          const int base = rs[iy] - bs[iy][0];
          k = max(c0, base + bs[iy][lz0]);
          e = min(c1, base + bs[iy][lz1]);
          ky = gy - (by0 + iy);
          ++iy;
        }
        if (k >= e) break;
        const int s = k - c0;
        const int kz0 = gz - bz0 - sbz[s];  // in [-1, Q]
        const R wxy = sw[s][0][kx] * sw[s][1][ky];
        const R wz0 = kz0 >= 0 ? sw[s][2][max(kz0, 0)] : R(0);
        const R wz1 = kz0 + 1 <= Q ? sw[s][2][min(kz0 + 1, Q)] : R(0);
        const R w0 = wxy * wz0, w1 = wxy * wz1;
#pragma unroll
        for (int pp = 0; pp < PB; ++pp) {
          const cplx<R> v = sq[s][pp];
          a0x[pp] += w0 * v.x;
          a0y[pp] += w0 * v.y;
          a1x[pp] += w1 * v.x;
          a1y[pp] += w1 * v.y;
        }
        ++k;
      }
    }
  }
  if (valid) {
    const int64_t node = (static_cast<int64_t>(gx) * g.n[1] + gy) * g.n[2] + gz;
#pragma unroll
    for (int pp = 0; pp < PB; ++pp)
      if (p0 + pp < P) grid[node * P + p0 + pp] = cmake<R>(a0x[pp], a0y[pp]);
    if (gz + 1 < g.n[2]) {
#pragma unroll
      for (int pp = 0; pp < PB; ++pp)
        if (p0 + pp < P) grid[(node + 1) * P + p0 + pp] = cmake<R>(a1x[pp], a1y[pp]);
    }
  }
}

// Projection from a node-major weight list (few planes): the transposed
// interpolation weights W^T as CSR by grid node, entries in increasing point
// order, built at plan time.  16 lanes per node add its entries and combine
// them by a fixed shuffle order.  With a node list (wnode, for grids mostly
// empty) only the listed nodes are visited and the grid is zeroed first;
// without one every node is visited and empty nodes write zero.
template <typename R>
__global__ void __launch_bounds__(256) k_spread_csr(const int64_t* __restrict__ wnode, int64_t nnodes,
                                                    const int64_t* __restrict__ wrow, const int32_t* __restrict__ widx,
                                                    const double* __restrict__ wval,
                                                    const cplx<R>* __restrict__ qint, int P,
                                                    cplx<R>* __restrict__ grid) {
  const int64_t i = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 4;
  const int sl = threadIdx.x & 15;
  if (i >= nnodes) return;  // all 16 lanes of a node leave together
  const int64_t node = wnode != nullptr ? wnode[i] : i;
  const int64_t j0 = wrow[i], j1 = wrow[i + 1];
  for (int p = 0; p < P; ++p) {
    double ar = 0.0, ai = 0.0;
    for (int64_t j = j0 + sl; j < j1; j += 16) {
      const double w = wval[j];
      const cplx<R> q = qint[static_cast<int64_t>(widx[j]) * P + p];
      ar += w * static_cast<double>(q.x);
      ai += w * static_cast<double>(q.y);
    }
    for (int off = 8; off > 0; off >>= 1) {
      ar += __shfl_xor(ar, off, 16);
      ai += __shfl_xor(ai, off, 16);
    }
    if (sl == 0) grid[node * P + p] = cmake<R>(static_cast<R>(ar), static_cast<R>(ai));
  }
}

template <typename R>
__global__ void __launch_bounds__(256) k_zero_grid(cplx<R>* __restrict__ grid, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += stride)
    grid[k] = cmake<R>(R(0), R(0));
}

// ---------------------------------------------------------------------------
// Step 3: interpolation from a grid to points (also the far zone's Step 3)
// ---------------------------------------------------------------------------

template <typename R, int Q, int PB>
__global__ void __launch_bounds__(256) k_interp(
    GridArgs g, const int32_t* __restrict__ s3, const double* __restrict__ w3, int64_t N,
    const cplx<R>* __restrict__ grid, int P, cplx<R>* __restrict__ uint, int accumulate) {
  int64_t m = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (m >= N) return;
  const int p0 = blockIdx.y * PB;
  double wx[Q + 1], wy[Q + 1], wz[Q + 1];
#pragma unroll
  for (int a = 0; a <= Q; ++a) {
    wx[a] = w3[a * N + m];
    wy[a] = w3[(Q + 1 + a) * N + m];
    wz[a] = w3[(2 * (Q + 1) + a) * N + m];
  }
  const int sx = s3[m], sy = s3[N + m], sz = s3[2 * N + m];
  double ax[PB], ay[PB];
#pragma unroll
  for (int pp = 0; pp < PB; ++pp) ax[pp] = ay[pp] = 0.0;
  for (int kx = 0; kx <= Q; ++kx) {
    for (int ky = 0; ky <= Q; ++ky) {
      const double wxy = wx[kx] * wy[ky];
      const int64_t row = (static_cast<int64_t>(sx + kx) * g.n[1] + (sy + ky)) * g.n[2] + sz;
#pragma unroll
      for (int kz = 0; kz <= Q; ++kz) {
        const double w = wxy * wz[kz];
#pragma unroll
        for (int pp = 0; pp < PB; ++pp) {
          if (p0 + pp < P) {
            cplx<R> v = grid[(row + kz) * P + p0 + pp];
            ax[pp] += w * static_cast<double>(v.x);
            ay[pp] += w * static_cast<double>(v.y);
          }
        }
      }
    }
  }
#pragma unroll
  for (int pp = 0; pp < PB; ++pp) {
    if (p0 + pp < P) {
      cplx<R>* o = uint + m * P + p0 + pp;
      cplx<R> r = cmake<R>(static_cast<R>(ax[pp]), static_cast<R>(ay[pp]));
      if (accumulate) r = cadd(*o, r);
      *o = r;
    }
  }
}

// Batched planes: the lanes of a wavefront cover LP planes x (64 / LP)
// points, so every stencil node is one contiguous, coalesced load of the
// node's planes; the point's weights are shared by its lanes.
template <typename R, int Q, int LP>
__global__ void __launch_bounds__(256) k_interp_lp(
    GridArgs g, const int32_t* __restrict__ s3, const double* __restrict__ w3, int64_t N,
    const cplx<R>* __restrict__ grid, int P, cplx<R>* __restrict__ uint, int accumulate) {
  constexpr int E = 64 / LP;
  const int lane = threadIdx.x & 63;
  const int e = lane / LP, pl = lane % LP;
  const int64_t m = (static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6)) * E + e;
  if (m >= N) return;
  double wx[Q + 1], wy[Q + 1], wz[Q + 1];
#pragma unroll
  for (int a = 0; a <= Q; ++a) {
    wx[a] = w3[a * N + m];
    wy[a] = w3[(Q + 1 + a) * N + m];
    wz[a] = w3[(2 * (Q + 1) + a) * N + m];
  }
  const int sx = s3[m], sy = s3[N + m], sz = s3[2 * N + m];
  for (int pc = 0; pc < P; pc += LP) {
    const int p = pc + pl;
    if (p >= P) continue;
    double ax = 0.0, ay = 0.0;
    for (int kx = 0; kx <= Q; ++kx) {
      for (int ky = 0; ky <= Q; ++ky) {
        const double wxy = wx[kx] * wy[ky];
        const cplx<R>* row = grid + ((static_cast<int64_t>(sx + kx) * g.n[1] + (sy + ky)) * g.n[2] + sz) * P + p;
        cplx<R> v[Q + 1];
#pragma unroll
        for (int kz = 0; kz <= Q; ++kz) v[kz] = row[static_cast<int64_t>(kz) * P];
#pragma unroll
        for (int kz = 0; kz <= Q; ++kz) {
          const double w = wxy * wz[kz];
          ax += w * static_cast<double>(v[kz].x);
          ay += w * static_cast<double>(v[kz].y);
        }
      }
    }
    cplx<R>* o = uint + m * P + p;
    cplx<R> r = cmake<R>(static_cast<R>(ax), static_cast<R>(ay));
    if (accumulate) r = cadd(*o, r);
    *o = r;
  }
}

// ---------------------------------------------------------------------------
// Step 2: FFT passes in LDS
// ---------------------------------------------------------------------------

__device__ inline int bitrev(int j, int logM) {
  return logM == 0 ? 0 : static_cast<int>(__brev(static_cast<unsigned>(j)) >> (32 - logM));
}

// Stages on T lines (T a power of 2) of length M held in LDS (line stride Ms), two radix-2 stages at a time
// (one radix-4 butterfly over elements base + {0, h, 2h, 3h}), a last
// radix-2 stage when log2 M is odd.  tw holds exp(-2 pi i k / M), k < M / 2
// (in LDS).  DIT: bit-reversed input -> natural output.  DIF: natural ->
// bit-reversed.  inverse selects the conjugated twiddles.
template <typename R>
__device__ inline cplx<R> twl(const cplx<R>* tw, int k, bool inverse) {
  cplx<R> w = tw[k];
  if (inverse) w.y = -w.y;
  return w;
}

template <typename R>
__device__ inline void lds_dit(cplx<R>* x, int T, int M, int Ms, int logM, const cplx<R>* tw, bool inverse) {
  // consecutive threads take consecutive lines (T is a power of 2; padded
  // line stride keeps them on different banks)
  const int logT = __ffs(T) - 1;
  int lh = 0;
  for (; lh + 1 < logM; lh += 2) {
    const int h = 1 << lh;
    const int nq = T * (M >> 2);
    for (int b = threadIdx.x; b < nq; b += blockDim.x) {
      const int t = b & (T - 1);
      const int k = b >> logT;
      const int pos = k & (h - 1);
      const int base = ((k >> lh) << (lh + 2)) + pos;
      cplx<R>* line = x + t * Ms;
      const cplx<R> w1 = twl(tw, pos << (logM - 1 - lh), inverse);
      const cplx<R> w2 = twl(tw, pos << (logM - 2 - lh), inverse);
      const cplx<R> w3 = twl(tw, (pos + h) << (logM - 2 - lh), inverse);
      const cplx<R> x0 = line[base], x1 = line[base + h], x2 = line[base + 2 * h], x3 = line[base + 3 * h];
      const cplx<R> b1 = cmul(x1, w1), d1 = cmul(x3, w1);
      const cplx<R> a = cadd(x0, b1), bb = csub(x0, b1), c = cadd(x2, d1), d = csub(x2, d1);
      const cplx<R> cw = cmul(c, w2), dw = cmul(d, w3);
      line[base] = cadd(a, cw);
      line[base + 2 * h] = csub(a, cw);
      line[base + h] = cadd(bb, dw);
      line[base + 3 * h] = csub(bb, dw);
    }
    __syncthreads();
  }
  if (lh < logM) {
    const int half = 1 << lh;
    const int nb = T * (M >> 1);
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
      const int t = b & (T - 1);
      const int k = b >> logT;
      const int pos = k & (half - 1);
      const int i0 = ((k >> lh) << (lh + 1)) + pos;
      const cplx<R> w = twl(tw, pos << (logM - 1 - lh), inverse);
      cplx<R>* line = x + t * Ms;
      const cplx<R> a = line[i0];
      const cplx<R> c = cmul(line[i0 + half], w);
      line[i0] = cadd(a, c);
      line[i0 + half] = csub(a, c);
    }
    __syncthreads();
  }
}

template <typename R>
__device__ inline void lds_dif(cplx<R>* x, int T, int M, int Ms, int logM, const cplx<R>* tw, bool inverse) {
  // consecutive threads take consecutive lines (T is a power of 2; padded
  // line stride keeps them on different banks)
  const int logT = __ffs(T) - 1;
  int lh = logM - 2;
  for (; lh >= 0; lh -= 2) {
    // stage lh + 1 then stage lh
    const int h = 1 << lh;
    const int nq = T * (M >> 2);
    for (int b = threadIdx.x; b < nq; b += blockDim.x) {
      const int t = b & (T - 1);
      const int k = b >> logT;
      const int pos = k & (h - 1);
      const int base = ((k >> lh) << (lh + 2)) + pos;
      cplx<R>* line = x + t * Ms;
      const cplx<R> w1 = twl(tw, pos << (logM - 1 - lh), inverse);
      const cplx<R> w2 = twl(tw, pos << (logM - 2 - lh), inverse);
      const cplx<R> w3 = twl(tw, (pos + h) << (logM - 2 - lh), inverse);
      const cplx<R> x0 = line[base], x1 = line[base + h], x2 = line[base + 2 * h], x3 = line[base + 3 * h];
      const cplx<R> a = cadd(x0, x2), c = cmul(csub(x0, x2), w2);
      const cplx<R> bb = cadd(x1, x3), d = cmul(csub(x1, x3), w3);
      line[base] = cadd(a, bb);
      line[base + h] = cmul(csub(a, bb), w1);
      line[base + 2 * h] = cadd(c, d);
      line[base + 3 * h] = cmul(csub(c, d), w1);
    }
    __syncthreads();
  }
  if (lh == -1) {
    // odd log2 M: the last stage (lh = 0) alone
    const int nb = T * (M >> 1);
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
      const int t = b & (T - 1);
      const int k = b >> logT;
      const int i0 = k << 1;
      const cplx<R> w = twl(tw, 0, inverse);
      cplx<R>* line = x + t * Ms;
      const cplx<R> a = line[i0];
      const cplx<R> c = line[i0 + 1];
      line[i0] = cadd(a, c);
      line[i0 + 1] = cmul(csub(a, c), w);
    }
    __syncthreads();
  }
}

// MODE 0: forward transform (bit-reversed load, DIT, natural store).
// MODE 1: inverse transform (natural load, DIF, bit-reversed store).
// MODE 2: forward DIT, multiply by spec (conjugated if conj_spec), inverse DIF.
template <typename R, int MODE>
__global__ void __launch_bounds__(256) k_fft_pass(const cplx<R>* in,
                                                  cplx<R>* out, FftPassDesc d,
                                                  const cplx<R>* __restrict__ tw,
                                                  const cplx<R>* __restrict__ spec, int conj_spec) {
  extern __shared__ unsigned char lds_raw[];
  cplx<R>* x = reinterpret_cast<cplx<R>*>(lds_raw);
  const int T = d.T, M = d.M, logM = d.logM;
  // LDS lines are padded by one element so that the column-strided load and
  // store phases do not all hit one bank
  const int Ms = M + 1;
  const int logT = __ffs(T) - 1;  // T is a power of 2
  cplx<R>* tws = x + static_cast<int64_t>(T) * Ms;  // [M / 2] twiddles
  for (int k = threadIdx.x; k < (M >> 1); k += blockDim.x) tws[k] = tw[k];
  int64_t outer = 0, c0 = 0, outer0 = 0;
  int nlines = T;
  if (d.contig) {
    outer0 = static_cast<int64_t>(blockIdx.x) * T;
    nlines = static_cast<int>(min<int64_t>(T, d.nouter - outer0));
  } else {
    const int64_t tiles = (d.ncols + T - 1) / T;
    outer = blockIdx.x / tiles;
    c0 = (blockIdx.x % tiles) * T;
    nlines = static_cast<int>(min<int64_t>(T, d.ncols - c0));
  }
  // load in batches of kFftLoadBatch elements per thread so that many loads
  // are in flight before any of them is stored to LDS
  constexpr int kFftLoadBatch = 8;
  for (int base = 0; base < T * M; base += blockDim.x * kFftLoadBatch) {
    cplx<R> v[kFftLoadBatch];
    int li[kFftLoadBatch];
#pragma unroll
    for (int u = 0; u < kFftLoadBatch; ++u) {
      const int idx = base + u * blockDim.x + threadIdx.x;
      v[u] = cmake<R>(R(0), R(0));
      li[u] = -1;
      if (idx < T * M) {
        int t, j;
        if (d.contig) {
          t = idx >> logM;
          j = idx & (M - 1);
        } else {
          t = idx & (T - 1);
          j = idx >> logT;
        }
        li[u] = t * Ms + ((MODE == 1) ? j : bitrev(j, logM));
        if (t < nlines && j < d.n_in) {
          const int64_t a = d.contig ? (outer0 + t) * d.in_outer + j * d.in_line
                                     : outer * d.in_outer + (c0 + t) * d.in_col + j * d.in_line;
          v[u] = in[a];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kFftLoadBatch; ++u)
      if (li[u] >= 0) x[li[u]] = v[u];
  }
  __syncthreads();
  if (MODE == 0 || MODE == 2) lds_dit<R>(x, T, M, Ms, logM, tws, false);
  if (MODE == 2) {
    // the lines of a block share spectrum values: consecutive threads take
    // consecutive lines at one frequency; the spectrum loads are issued
    // kFftLoadBatch per thread before they are used
    for (int base = 0; base < T * M; base += blockDim.x * kFftLoadBatch) {
      cplx<R> s[kFftLoadBatch];
      int li[kFftLoadBatch];
#pragma unroll
      for (int u = 0; u < kFftLoadBatch; ++u) {
        const int idx = base + u * blockDim.x + threadIdx.x;
        const int k = idx >> logT;
        const int t = idx & (T - 1);
        li[u] = (idx < T * M && t < nlines) ? t * Ms + k : -1;
        s[u] = li[u] >= 0 ? spec[static_cast<int64_t>(k) * d.spec_line + ((c0 + t) / d.spec_div) * d.spec_col]
                          : cmake<R>(R(0), R(0));
      }
#pragma unroll
      for (int u = 0; u < kFftLoadBatch; ++u) {
        if (li[u] < 0) continue;
        cplx<R> sv = s[u];
        if (conj_spec) sv.y = -sv.y;
        x[li[u]] = cmul(x[li[u]], sv);
      }
    }
    __syncthreads();
  }
  if (MODE == 1 || MODE == 2) lds_dif<R>(x, T, M, Ms, logM, tws, true);
  for (int idx = threadIdx.x; idx < T * d.n_out; idx += blockDim.x) {
    int t, j;
    if (d.contig) {
      t = idx / d.n_out;
      j = idx - t * d.n_out;
    } else {
      t = idx & (T - 1);
      j = idx >> logT;
    }
    if (t >= nlines) continue;
    const int pos = (MODE == 0) ? j : bitrev(j, logM);
    int64_t a = d.contig ? (outer0 + t) * d.out_outer + j * d.out_line
                         : outer * d.out_outer + (c0 + t) * d.out_col + j * d.out_line;
    out[a] = x[t * Ms + pos];
  }
}

// Strided passes with the line length M = A B in registers (Cooley-Tukey in
// four steps): with n = B n1 + n2 and k = k1 + A k2,
//   X[k1 + A k2] = sum_n2 W_B^(n2 k2) W_M^(n2 k1) sum_n1 W_A^(n1 k1) x[B n1 + n2].
// A group of TL = min(A, B) threads owns a line: first each thread takes
// B / TL values of n2 and transforms its A points in registers, applies the
// twiddles W_M^(n2 k1), and the line is exchanged once through LDS; then each
// thread takes A / TL values of k1 and transforms the B points.  The inverse
// runs the same steps backwards (the k1-owned layout after a forward transform
// is the one the inverse starts from, so the fused pass needs no exchange
// between the spectrum multiply and the inverse).  Consecutive threads take
// consecutive lines, so every global load and store is a run of T columns.
// Natural order in and out, forward exp(-2 pi i / M), unscaled inverse, as the
// LDS-stage kernel above.
// cos(pi k / 16) and sin(pi k / 16), k = 0..16: the twiddles inside the
// register transforms (lines of at most 32 values), from their Taylor series
// at compile time, so that every butterfly's factor is an immediate and the
// factors 1 and -i cost no multiplications
constexpr double ct_sin(double x) {
  double term = x, sum = x;
  for (int n = 1; n < 24; ++n) {
    term *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double ct_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 24; ++n) {
    term *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
    sum += term;
  }
  return sum;
}
struct RegTwiddles {
  double c[17], s[17];
  constexpr RegTwiddles() : c(), s() {
    for (int k = 0; k <= 16; ++k) {
      c[k] = ct_cos(3.14159265358979323846 * k / 16.0);
      s[k] = ct_sin(3.14159265358979323846 * k / 16.0);
    }
  }
};
constexpr RegTwiddles kRegTw{};

template <typename R, int L>
__device__ inline void reg_dft(cplx<R>* v, const cplx<R>* tws, int twstride, bool inverse) {
  static_assert(L <= 32, "register lines of at most 32 values");
  (void)tws;
  (void)twstride;
  // bit-reversal permutation (compile-time indices)
#pragma unroll
  for (int i = 0; i < L; ++i) {
    int j = 0;
#pragma unroll
    for (int b = 1, m = L >> 1; b < L; b <<= 1, m >>= 1)
      if (i & b) j |= m;
    if (j > i) {
      const cplx<R> tmp = v[i];
      v[i] = v[j];
      v[j] = tmp;
    }
  }
#pragma unroll
  for (int s = 1; s < L; s <<= 1) {
#pragma unroll
    for (int k = 0; k < L; k += 2 * s) {
#pragma unroll
      for (int j = 0; j < s; ++j) {
        cplx<R> b = v[k + j + s];
        // factor exp(-+ i pi e / 16) with e = 16 j / s
        const int e = 16 * j / s;
        if (e == 8) {
          b = inverse ? cmake<R>(-b.y, b.x) : cmake<R>(b.y, -b.x);
        } else if (e != 0) {
          const R c = static_cast<R>(kRegTw.c[e]);
          const R sn = static_cast<R>(kRegTw.s[e]);
          b = cmul(b, cmake<R>(c, inverse ? sn : -sn));
        }
        const cplx<R> a = v[k + j];
        v[k + j] = cadd(a, b);
        v[k + j + s] = csub(a, b);
      }
    }
  }
}

// W_M^e (conjugated for the inverse) from the half table exp(-2 pi i k / M), k < M / 2
template <typename R, int M>
__device__ inline cplx<R> tw_full(const cplx<R>* tws, int e, bool inverse) {
  e &= M - 1;
  cplx<R> w = tws[e & (M / 2 - 1)];
  if (e >= M / 2) {
    w.x = -w.x;
    w.y = -w.y;
  }
  if (inverse) w.y = -w.y;
  return w;
}

template <typename R, int MODE, int A, int B, int NTH>
__global__ void __launch_bounds__(NTH) k_fft_reg(const cplx<R>* in, cplx<R>* out, FftPassDesc d,
                                                 const cplx<R>* __restrict__ tw, const cplx<R>* __restrict__ spec,
                                                 int conj_spec) {
  constexpr int M = A * B;
  constexpr int TL = A < B ? A : B;  // threads per line
  constexpr int T = NTH / TL;        // lines per block
  constexpr int E1 = B / TL;         // length-A transforms per thread
  constexpr int E3 = A / TL;         // length-B transforms per thread
  constexpr int E = M / TL;          // values per thread
  constexpr int LS = M + 1;          // LDS line stride
  extern __shared__ unsigned char lds_raw[];
  cplx<R>* xs = reinterpret_cast<cplx<R>*>(lds_raw);  // [T][LS]
  cplx<R>* tws = xs + T * LS;                         // [M / 2]
  for (int k = threadIdx.x; k < M / 2; k += NTH) tws[k] = tw[k];
  const int t = threadIdx.x % T, r = threadIdx.x / T;
  const int64_t tiles = (d.ncols + T - 1) / T;
  const int64_t outer = blockIdx.x / tiles;
  const int64_t col = (blockIdx.x % tiles) * T + t;
  const bool line_ok = col < d.ncols;
  const cplx<R>* src = in + outer * d.in_outer + col * d.in_col;
  cplx<R>* dst = out + outer * d.out_outer + col * d.out_col;
  cplx<R> v[E];
  if (MODE == 0 || MODE == 2) {
    // x[B n1 + n2] for this thread's n2 = r + TL e1
#pragma unroll
    for (int e1 = 0; e1 < E1; ++e1)
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) {
        const int j = B * n1 + r + TL * e1;
        v[e1 * A + n1] = (line_ok && j < d.n_in) ? src[j * d.in_line] : cmake<R>(R(0), R(0));
      }
  } else {
    // X[k1 + A k2] for this thread's k1 = r + TL e3
#pragma unroll
    for (int e3 = 0; e3 < E3; ++e3)
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) {
        const int k = r + TL * e3 + A * k2;
        v[e3 * B + k2] = (line_ok && k < d.n_in) ? src[k * d.in_line] : cmake<R>(R(0), R(0));
      }
  }
  __syncthreads();  // twiddle table
  cplx<R>* xl = xs + t * LS;
  if (MODE == 0 || MODE == 2) {
#pragma unroll
    for (int e1 = 0; e1 < E1; ++e1) {
      const int n2 = r + TL * e1;
      reg_dft<R, A>(v + e1 * A, tws, M / A, false);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) xl[k1 * B + n2] = cmul(v[e1 * A + k1], tw_full<R, M>(tws, n2 * k1, false));
    }
    __syncthreads();
#pragma unroll
    for (int e3 = 0; e3 < E3; ++e3) {
      const int k1 = r + TL * e3;
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) v[e3 * B + n2] = xl[k1 * B + n2];
      reg_dft<R, B>(v + e3 * B, tws, M / B, false);
    }
    if (MODE == 2) {
      // spectrum of every k = k1 + A k2 held here; planes share a value
      const int64_t sc = (col / d.spec_div) * d.spec_col;
      cplx<R> sv[E];
#pragma unroll
      for (int e3 = 0; e3 < E3; ++e3)
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2)
          sv[e3 * B + k2] = line_ok ? spec[static_cast<int64_t>(r + TL * e3 + A * k2) * d.spec_line + sc]
                                    : cmake<R>(R(0), R(0));
#pragma unroll
      for (int i = 0; i < E; ++i) {
        cplx<R> w = sv[i];
        if (conj_spec) w.y = -w.y;
        v[i] = cmul(v[i], w);
      }
      __syncthreads();  // the LDS lines are rewritten below
    }
  }
  if (MODE == 0) {
#pragma unroll
    for (int e3 = 0; e3 < E3; ++e3)
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) {
        const int k = r + TL * e3 + A * k2;
        if (line_ok && k < d.n_out) dst[k * d.out_line] = v[e3 * B + k2];
      }
    return;
  }
  // inverse: x[n2 + B n1] = sum_k1 W_A^-(n1 k1) W_M^-(n2 k1) sum_k2 W_B^-(n2 k2) X[k1 + A k2]
#pragma unroll
  for (int e3 = 0; e3 < E3; ++e3) {
    const int k1 = r + TL * e3;
    reg_dft<R, B>(v + e3 * B, tws, M / B, true);
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) xl[k1 * B + n2] = cmul(v[e3 * B + n2], tw_full<R, M>(tws, n2 * k1, true));
  }
  __syncthreads();
#pragma unroll
  for (int e1 = 0; e1 < E1; ++e1) {
    const int n2 = r + TL * e1;
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) v[e1 * A + k1] = xl[k1 * B + n2];
    reg_dft<R, A>(v + e1 * A, tws, M / A, true);
#pragma unroll
    for (int n1 = 0; n1 < A; ++n1) {
      const int j = n2 + B * n1;
      if (line_ok && j < d.n_out) dst[j * d.out_line] = v[e1 * A + n1];
    }
  }
}

// ---------------------------------------------------------------------------
// plan time: near-zone table G^p_near at node offsets, circularly embedded
// ---------------------------------------------------------------------------

__global__ void k_near_table(cplx<double>* __restrict__ T, NearTableArgs a) {
  int64_t total = static_cast<int64_t>(a.M[0]) * a.M[1] * a.M[2];
  int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  int i[3];
  i[2] = static_cast<int>(idx % a.M[2]);
  i[1] = static_cast<int>((idx / a.M[2]) % a.M[1]);
  i[0] = static_cast<int>(idx / (static_cast<int64_t>(a.M[1]) * a.M[2]));
  int e[3];
  bool inside = true;
  for (int c = 0; c < 3; ++c) {
    e[c] = i[c] < a.n[c] ? i[c] : i[c] - a.M[c];
    if (e[c] > a.n[c] - 1 || e[c] < -(a.n[c] - 1)) inside = false;
  }
  double sr = 0.0, si = 0.0;
  if (inside) {
    for (int k = 0; k < a.nimg; ++k) {
      int f[3];
      for (int c = 0; c < 3; ++c) f[c] = e[c] - a.img[3 * k + c] * a.nint[c];
      if (f[0] == 0 && f[1] == 0 && f[2] == 0) continue;  // singular term set to 0
      double dx = f[0] * a.h[0], dy = f[1] * a.h[1], dz = f[2] * a.h[2];
      double r = sqrt(dx * dx + dy * dy + dz * dz);
      double s, c;
      sincos(a.k0 * r, &s, &c);
      // a lossy k0 = k0 + j k0_im adds the factor exp(k0_im r)
      double inv = (a.k0_im != 0.0 ? exp(a.k0_im * r) : 1.0) / (4.0 * M_PI * r);
      // phase * exp(-j k0 r) / (4 pi r)
      double gr = c * inv, gi = -s * inv;
      sr += a.phase[2 * k] * gr - a.phase[2 * k + 1] * gi;
      si += a.phase[2 * k] * gi + a.phase[2 * k + 1] * gr;
    }
  }
  T[idx] = cmake<double>(sr, si);
}

template <typename R>
__global__ void k_scale_convert(const cplx<double>* __restrict__ in, cplx<R>* __restrict__ out,
                                int64_t n, double s) {
  int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  cplx<double> v = in[idx];
  out[idx] = cmake<R>(static_cast<R>(v.x * s), static_cast<R>(v.y * s));
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline unsigned blocks_for(int64_t n, int bs) { return static_cast<unsigned>((n + bs - 1) / bs); }

// Block size of the per-point / per-node kernels for few planes (projection
// through the weight CSR, interpolation): one wavefront, so they are
// scheduled on compute units the concurrent correction keeps nearly full.
constexpr int kPointBlock = 64;

template <typename R>
void launch_pack(const void* qu, void* qint, const int32_t* perm, int64_t N, int nrhs, int P,
                 bool real_in, bool use_perm, hipStream_t st) {
  if (P >= 4) {
    dim3 gr(static_cast<unsigned>((N + kTpPts - 1) / kTpPts), static_cast<unsigned>((P + kTpPl - 1) / kTpPl));
    if (real_in)
      hipLaunchKernelGGL((k_pack_tiled<R, true>), gr, dim3(256), 0, st, qu, static_cast<cplx<R>*>(qint), perm, N,
                         nrhs, P, use_perm ? 1 : 0);
    else
      hipLaunchKernelGGL((k_pack_tiled<R, false>), gr, dim3(256), 0, st, qu, static_cast<cplx<R>*>(qint), perm, N,
                         nrhs, P, use_perm ? 1 : 0);
    return;
  }
  unsigned nb = blocks_for(N * P, 256);
  if (real_in)
    hipLaunchKernelGGL((k_pack<R, true>), dim3(nb), dim3(256), 0, st, qu,
                       static_cast<cplx<R>*>(qint), perm, N, nrhs, P, use_perm ? 1 : 0);
  else
    hipLaunchKernelGGL((k_pack<R, false>), dim3(nb), dim3(256), 0, st, qu,
                       static_cast<cplx<R>*>(qint), perm, N, nrhs, P, use_perm ? 1 : 0);
}

template <typename R>
static PartPtrs<R> part_ptrs(const void* a, const void* b, const void* c, DiagTerm diag = DiagTerm()) {
  PartPtrs<R> s;
  s.a = static_cast<const cplx<R>*>(a);
  s.b = static_cast<const cplx<R>*>(b);
  s.c = static_cast<const cplx<R>*>(c);
  s.self = static_cast<const cplx<R>*>(diag.in);
  s.cr = static_cast<R>(diag.re);
  s.ci = static_cast<R>(diag.im);
  return s;
}

template <typename R>
void launch_unpack(const void* u_near, const void* u_corr, const void* u_far, void* uu, const int32_t* perm,
                   int64_t N, int nrhs, int P, bool real_out, bool use_perm, const double* mean, hipStream_t st,
                   DiagTerm diag) {
  PartPtrs<R> s = part_ptrs<R>(u_near, u_corr, u_far, diag);
  if (P >= 4) {
    dim3 gr(static_cast<unsigned>((N + kTpPts - 1) / kTpPts), static_cast<unsigned>((P + kTpPl - 1) / kTpPl));
    if (real_out)
      hipLaunchKernelGGL((k_unpack_tiled<R, true>), gr, dim3(256), 0, st, s, uu, perm, N, nrhs, P, use_perm ? 1 : 0,
                         mean);
    else
      hipLaunchKernelGGL((k_unpack_tiled<R, false>), gr, dim3(256), 0, st, s, uu, perm, N, nrhs, P,
                         use_perm ? 1 : 0, mean);
    return;
  }
  unsigned nb = blocks_for(N * P, 256);
  if (real_out)
    hipLaunchKernelGGL((k_unpack<R, true>), dim3(nb), dim3(256), 0, st, s, uu, perm, N, nrhs, P, use_perm ? 1 : 0,
                       mean);
  else
    hipLaunchKernelGGL((k_unpack<R, false>), dim3(nb), dim3(256), 0, st, s, uu, perm, N, nrhs, P,
                       use_perm ? 1 : 0, mean);
}

int64_t plane_sums_chunks(int64_t N) { return (N + kPlaneSumChunk - 1) / kPlaneSumChunk; }

template <typename R>
void launch_plane_sums(const void* a, const void* b, const void* c, int64_t N, int P, double* work, double* out,
                       hipStream_t st, DiagTerm diag) {
  const int64_t nch = plane_sums_chunks(N);
  hipLaunchKernelGGL((k_plane_sums_part<R>), dim3(static_cast<unsigned>(nch), static_cast<unsigned>((P + 63) / 64)),
                     dim3(256), 0, st, part_ptrs<R>(a, b, c, diag), N, P, work);
  hipLaunchKernelGGL(k_plane_sums_final, dim3(static_cast<unsigned>((P + 63) / 64)), dim3(64), 0, st, work, nch, P,
                     out);
}

void launch_check_neutral(const double* sums, int P, double tol, int* status, hipStream_t st) {
  hipLaunchKernelGGL(k_check_neutral, dim3(1), dim3(64), 0, st, sums, P, tol, status);
}

void launch_mean_from_sums(const double* sums, int P, int64_t N, double* mean, hipStream_t st) {
  hipLaunchKernelGGL(k_mean_from_sums, dim3(1), dim3(64), 0, st, sums, P, 1.0 / static_cast<double>(N), mean);
}

#define FFTPIM_PB_DISPATCH(P, CALL) \
  do {                               \
    if ((P) >= 8) {                  \
      constexpr int PB = 8;          \
      CALL;                          \
    } else if ((P) >= 4) {           \
      constexpr int PB = 4;          \
      CALL;                          \
    } else if ((P) >= 2) {           \
      constexpr int PB = 2;          \
      CALL;                          \
    } else {                         \
      constexpr int PB = 1;          \
      CALL;                          \
    }                                \
  } while (0)

template <typename R, int Q>
static void spread_q(const GridArgs& g, const int32_t* box_start, const int32_t* s3, const double* u3,
                     int64_t N, const void* qint, int P, void* grid, hipStream_t st) {
  if (P >= 16) {
    // many planes: the own-list form
    const unsigned otiles = static_cast<unsigned>(((g.n[0] + kOwnTX - 1) / kOwnTX) *
                                                  ((g.n[1] + kOwnTY - 1) / kOwnTY) *
                                                  ((g.n[2] + kOwnTZ - 1) / kOwnTZ));
    dim3 gr(otiles, (P + OwnCfg<R>::PB - 1) / OwnCfg<R>::PB);
    hipLaunchKernelGGL((k_spread_own<R, Q>), gr, dim3(256), 0, st, g, box_start, s3, u3, N,
                       static_cast<const cplx<R>*>(qint), P, static_cast<cplx<R>*>(grid));
    return;
  }
  const unsigned tiles = static_cast<unsigned>(((g.n[0] + kSpreadTX - 1) / kSpreadTX) *
                                               ((g.n[1] + kSpreadTY - 1) / kSpreadTY) *
                                               ((g.n[2] + kSpreadTZ - 1) / kSpreadTZ));
#define FFTPIM_SPREAD_PB(PBV)                                                                              \
  do {                                                                                                     \
    dim3 gr(tiles, (P + PBV - 1) / PBV);                                                                   \
    hipLaunchKernelGGL((k_spread_near<R, Q, PBV>), gr, dim3(256), 0, st, g, box_start, s3, u3, N,          \
                       static_cast<const cplx<R>*>(qint), P, static_cast<cplx<R>*>(grid));                 \
  } while (0)
  FFTPIM_PB_DISPATCH(P, FFTPIM_SPREAD_PB(PB));
#undef FFTPIM_SPREAD_PB
}

template <typename R>
void launch_spread_csr(const int64_t* wnode, int64_t nnodes, const int64_t* wrow, const int32_t* widx,
                       const double* wval, int64_t n3, const void* qint, int P, void* grid, hipStream_t st) {
  if (wnode != nullptr) {
    const int64_t nz = n3 * P;
    hipLaunchKernelGGL((k_zero_grid<R>), dim3(static_cast<unsigned>(std::min<int64_t>(blocks_for(nz, 256), 65536))),
                       dim3(256), 0, st, static_cast<cplx<R>*>(grid), nz);
  }
  if (nnodes > 0)
    hipLaunchKernelGGL((k_spread_csr<R>), dim3(blocks_for(nnodes * 16, kPointBlock)), dim3(kPointBlock), 0, st,
                       wnode, nnodes, wrow, widx, wval, static_cast<const cplx<R>*>(qint), P,
                       static_cast<cplx<R>*>(grid));
}

template <typename R>
int launch_spread_near(int q, const GridArgs& g, const int32_t* box_start, const int32_t* s3, const double* u3,
                       int64_t N, const void* qint, int P, void* grid, hipStream_t st) {
  switch (q) {
    case 1: spread_q<R, 1>(g, box_start, s3, u3, N, qint, P, grid, st); break;
    case 2: spread_q<R, 2>(g, box_start, s3, u3, N, qint, P, grid, st); break;
    case 3: spread_q<R, 3>(g, box_start, s3, u3, N, qint, P, grid, st); break;
    case 4: spread_q<R, 4>(g, box_start, s3, u3, N, qint, P, grid, st); break;
    case 5: spread_q<R, 5>(g, box_start, s3, u3, N, qint, P, grid, st); break;
    case 6: spread_q<R, 6>(g, box_start, s3, u3, N, qint, P, grid, st); break;
    case 7: spread_q<R, 7>(g, box_start, s3, u3, N, qint, P, grid, st); break;
    case 8: spread_q<R, 8>(g, box_start, s3, u3, N, qint, P, grid, st); break;
    default: return FFTPIM_ERR_UNSUPPORTED;
  }
  return FFTPIM_OK;
}

template <typename R, int Q>
static void interp_q(const GridArgs& g, const int32_t* s3, const double* u3, int64_t N, const void* grid,
                     int P, void* uint, bool acc, hipStream_t st) {
  if (P >= 8) {
    // lanes over planes: LP planes x 64 / LP points per wavefront, 4 wavefronts per block
#define FFTPIM_INTERP_LP(LPV)                                                                              \
  do {                                                                                                     \
    const int64_t pts_per_block = 4 * (64 / LPV);                                                          \
    hipLaunchKernelGGL((k_interp_lp<R, Q, LPV>), dim3(static_cast<unsigned>((N + pts_per_block - 1) / pts_per_block)), \
                       dim3(256), 0, st, g, s3, u3, N, static_cast<const cplx<R>*>(grid), P,               \
                       static_cast<cplx<R>*>(uint), acc ? 1 : 0);                                          \
  } while (0)
    if (P <= 16)
      FFTPIM_INTERP_LP(16);
    else if (P <= 32)
      FFTPIM_INTERP_LP(32);
    else
      FFTPIM_INTERP_LP(64);
#undef FFTPIM_INTERP_LP
    return;
  }
  FFTPIM_PB_DISPATCH(P, {
    dim3 gr(blocks_for(N, kPointBlock), (P + PB - 1) / PB);
    hipLaunchKernelGGL((k_interp<R, Q, PB>), gr, dim3(kPointBlock), 0, st, g, s3, u3, N,
                       static_cast<const cplx<R>*>(grid), P, static_cast<cplx<R>*>(uint), acc ? 1 : 0);
  });
}

template <typename R>
int launch_interp(int q, const GridArgs& g, const int32_t* s3, const double* u3, int64_t N, const void* grid,
                  int P, void* uint, bool acc, hipStream_t st) {
  switch (q) {
    case 1: interp_q<R, 1>(g, s3, u3, N, grid, P, uint, acc, st); break;
    case 2: interp_q<R, 2>(g, s3, u3, N, grid, P, uint, acc, st); break;
    case 3: interp_q<R, 3>(g, s3, u3, N, grid, P, uint, acc, st); break;
    case 4: interp_q<R, 4>(g, s3, u3, N, grid, P, uint, acc, st); break;
    case 5: interp_q<R, 5>(g, s3, u3, N, grid, P, uint, acc, st); break;
    case 6: interp_q<R, 6>(g, s3, u3, N, grid, P, uint, acc, st); break;
    case 7: interp_q<R, 7>(g, s3, u3, N, grid, P, uint, acc, st); break;
    case 8: interp_q<R, 8>(g, s3, u3, N, grid, P, uint, acc, st); break;
    case 9: interp_q<R, 9>(g, s3, u3, N, grid, P, uint, acc, st); break;
    default: return FFTPIM_ERR_UNSUPPORTED;
  }
  return FFTPIM_OK;
}

template <typename R, int A, int B, int NTH>
static void fft_reg_n(int mode, const cplx<R>* i, cplx<R>* o, const FftPassDesc& d, const cplx<R>* t,
                      const cplx<R>* s, bool conj_spec, hipStream_t st) {
  constexpr int M = A * B, TL = A < B ? A : B, T = NTH / TL;
  const unsigned nblocks = static_cast<unsigned>(d.nouter * ((d.ncols + T - 1) / T));
  const size_t lds = (static_cast<size_t>(T) * (M + 1) + M / 2) * sizeof(cplx<R>);
  if (mode == 0)
    hipLaunchKernelGGL((k_fft_reg<R, 0, A, B, NTH>), dim3(nblocks), dim3(NTH), lds, st, i, o, d, t, s, 0);
  else if (mode == 1)
    hipLaunchKernelGGL((k_fft_reg<R, 1, A, B, NTH>), dim3(nblocks), dim3(NTH), lds, st, i, o, d, t, s, 0);
  else
    hipLaunchKernelGGL((k_fft_reg<R, 2, A, B, NTH>), dim3(nblocks), dim3(NTH), lds, st, i, o, d, t, s,
                       conj_spec ? 1 : 0);
}

// 256 threads per block, or 128 where the lines of 256 threads would need
// more than 64 KB of LDS
template <typename R, int A, int B>
static bool fft_reg(int mode, const cplx<R>* i, cplx<R>* o, const FftPassDesc& d, const cplx<R>* t,
                    const cplx<R>* s, bool conj_spec, hipStream_t st) {
  constexpr int M = A * B, TL = A < B ? A : B;
  constexpr size_t lds256 = (static_cast<size_t>(256 / TL) * (M + 1) + M / 2) * sizeof(cplx<R>);
  constexpr size_t lds128 = (static_cast<size_t>(128 / TL) * (M + 1) + M / 2) * sizeof(cplx<R>);
  if (lds256 <= 65536)
    fft_reg_n<R, A, B, 256>(mode, i, o, d, t, s, conj_spec, st);
  else if (lds128 <= 65536)
    fft_reg_n<R, A, B, 128>(mode, i, o, d, t, s, conj_spec, st);
  else
    return false;
  return true;
}

// Register transforms for strided FP32 passes of length 16..512; other passes
// (lines contiguous in memory, FP64) go through the LDS-stage kernel.
template <typename R>
static bool launch_fft_reg(int mode, const cplx<R>* i, cplx<R>* o, const FftPassDesc& d, const cplx<R>* t,
                           const cplx<R>* s, bool conj_spec, hipStream_t st) {
  if constexpr (sizeof(R) != 4) {
    // FP64 lines of 16 values per thread cost occupancy; measured slower
    // than the LDS stages on the FP64 workloads
    return false;
  } else {
  if (d.contig) return false;
  switch (d.M) {
    case 16: return fft_reg<R, 4, 4>(mode, i, o, d, t, s, conj_spec, st);
    case 32: return fft_reg<R, 8, 4>(mode, i, o, d, t, s, conj_spec, st);
    case 64: return fft_reg<R, 8, 8>(mode, i, o, d, t, s, conj_spec, st);
    case 128: return fft_reg<R, 16, 8>(mode, i, o, d, t, s, conj_spec, st);
    case 256: return fft_reg<R, 16, 16>(mode, i, o, d, t, s, conj_spec, st);
    case 512: return fft_reg<R, 16, 32>(mode, i, o, d, t, s, conj_spec, st);
    default: return false;
  }
  }
}

template <typename R>
void launch_fft_pass(int mode, const void* in, void* out, const FftPassDesc& d, const void* tw,
                     const void* spec, bool conj_spec, hipStream_t st) {
  if (launch_fft_reg<R>(mode, static_cast<const cplx<R>*>(in), static_cast<cplx<R>*>(out), d,
                        static_cast<const cplx<R>*>(tw), static_cast<const cplx<R>*>(spec), conj_spec, st))
    return;
  unsigned nblocks = d.contig ? blocks_for(d.nouter, d.T)
                              : static_cast<unsigned>(d.nouter * ((d.ncols + d.T - 1) / d.T));
  size_t lds = (static_cast<size_t>(d.T) * (d.M + 1) + d.M / 2) * sizeof(cplx<R>);
  const cplx<R>* i = static_cast<const cplx<R>*>(in);
  cplx<R>* o = static_cast<cplx<R>*>(out);
  const cplx<R>* t = static_cast<const cplx<R>*>(tw);
  const cplx<R>* s = static_cast<const cplx<R>*>(spec);
  if (mode == 0)
    hipLaunchKernelGGL((k_fft_pass<R, 0>), dim3(nblocks), dim3(256), lds, st, i, o, d, t, s, 0);
  else if (mode == 1)
    hipLaunchKernelGGL((k_fft_pass<R, 1>), dim3(nblocks), dim3(256), lds, st, i, o, d, t, s, 0);
  else
    hipLaunchKernelGGL((k_fft_pass<R, 2>), dim3(nblocks), dim3(256), lds, st, i, o, d, t, s,
                       conj_spec ? 1 : 0);
}

void launch_near_table(void* T, const NearTableArgs& a, hipStream_t st) {
  int64_t total = static_cast<int64_t>(a.M[0]) * a.M[1] * a.M[2];
  hipLaunchKernelGGL(k_near_table, dim3(blocks_for(total, 256)), dim3(256), 0, st,
                     static_cast<cplx<double>*>(T), a);
}

template <typename R>
void launch_scale_convert(const void* in, void* out, int64_t n, double s, hipStream_t st) {
  hipLaunchKernelGGL((k_scale_convert<R>), dim3(blocks_for(n, 256)), dim3(256), 0, st,
                     static_cast<const cplx<double>*>(in), static_cast<cplx<R>*>(out), n, s);
}

// explicit instantiations
#define FFTPIM_INST_GRID(R)                                                                              \
  template void launch_pack<R>(const void*, void*, const int32_t*, int64_t, int, int, bool, bool,        \
                               hipStream_t);                                                             \
  template void launch_unpack<R>(const void*, const void*, const void*, void*, const int32_t*, int64_t,  \
                                 int, int, bool, bool, const double*, hipStream_t, DiagTerm);            \
  template void launch_plane_sums<R>(const void*, const void*, const void*, int64_t, int, double*, double*, \
                                     hipStream_t, DiagTerm);                                             \
  template void launch_spread_csr<R>(const int64_t*, int64_t, const int64_t*, const int32_t*, const double*, \
                                     int64_t, const void*, int, void*, hipStream_t);                                                \
  template int launch_spread_near<R>(int, const GridArgs&, const int32_t*, const int32_t*, const double*, \
                                     int64_t, const void*, int, void*, hipStream_t);                     \
  template int launch_interp<R>(int, const GridArgs&, const int32_t*, const double*, int64_t,            \
                                const void*, int, void*, bool, hipStream_t);                             \
  template void launch_fft_pass<R>(int, const void*, void*, const FftPassDesc&, const void*, const void*, \
                                   bool, hipStream_t);                                                   \
  template void launch_scale_convert<R>(const void*, void*, int64_t, double, hipStream_t);

FFTPIM_INST_GRID(double)
FFTPIM_INST_GRID(float)

}  // namespace fftpim
