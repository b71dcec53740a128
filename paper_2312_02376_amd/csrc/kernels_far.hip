// Far zone, Sec. 3.2.
//   Step 1 (Eq. (projection)): projection onto the sparse source grid, done
//     atomic-free in two stages: every far box sums the weighted amplitudes
//     of its points into its own (qf+1)^3 stencil patch ("moments"), then
//     every grid node gathers the patches that cover it.
//   Step 2 (Eq. (8)): the dense grid sum u_g[m'] = sum_n' K[m', n'] q_g[n'].
//     K is shift invariant, K[m', n'] = G^p_far((m' - n') h - h/2), so its
//     tiles are generated from the (2 nf - 1)^3 offset table instead of being
//     stored (the table stays in L2).  The conjugate transpose uses
//     conj(K[n', m']) from the same table.
//   Step 3 (Eq. (interpolation)): the generic grid-to-point interpolation.
#include <algorithm>

#include "kernels.h"

namespace fftpim {

// One block per far box, one thread per (x, y) pair of local stencil nodes
// looping over the qf+1 z nodes (the x-y weight product is formed once per
// point and reused along z).  The box's points are staged through LDS in
// chunks with their 1D weights.  A block is one or two wavefronts, so the
// kernel finds room on compute units that the concurrent correction keeps
// nearly full.
constexpr int kMomChunk = 64;

// Block size of the elementwise far-zone kernels (gather, dense sum for few
// planes, split reduction): one wavefront, so they are scheduled on compute
// units the concurrent correction keeps nearly full.
constexpr int kFarBlock = 64;

template <typename R, int QF, int PB>
__global__ void __launch_bounds__(128) k_far_moments(const int32_t* __restrict__ fbox_start,
                                                     const int32_t* __restrict__ fperm,
                                                     const double* __restrict__ w3, int64_t N,
                                                     const cplx<R>* __restrict__ qint, int P,
                                                     cplx<R>* __restrict__ mom) {
  constexpr int K1 = QF + 1;
  constexpr int K = K1 * K1 * K1;
  constexpr int CH = kMomChunk;
  __shared__ double sw[CH][3][K1];
  __shared__ cplx<R> sq[CH][PB];
  const int t = threadIdx.x;
  const int64_t b = blockIdx.x;
  const int p0 = blockIdx.y * PB;
  const bool own = t < K1 * K1;
  const int kx = t / K1, ky = t % K1;
  double ar[K1][PB], ai[K1][PB];
#pragma unroll
  for (int c = 0; c < K1; ++c)
#pragma unroll
    for (int pp = 0; pp < PB; ++pp) ar[c][pp] = ai[c][pp] = 0.0;
  const int j0 = fbox_start[b], j1 = fbox_start[b + 1];
  for (int base = j0; base < j1; base += CH) {
    __syncthreads();
    for (int i = t; i < CH; i += blockDim.x) {
      if (base + i < j1) {
        const int n = fperm[base + i];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int a = 0; a < K1; ++a) sw[i][c][a] = w3[(c * K1 + a) * N + n];
#pragma unroll
        for (int pp = 0; pp < PB; ++pp)
          sq[i][pp] = (p0 + pp < P) ? qint[static_cast<int64_t>(n) * P + p0 + pp] : cmake<R>(R(0), R(0));
      }
    }
    __syncthreads();
    const int cnt = min(CH, j1 - base);
    if (own) {
      for (int i = 0; i < cnt; ++i) {
        const double wxy = sw[i][0][kx] * sw[i][1][ky];
        double qr[PB], qi[PB];
#pragma unroll
        for (int pp = 0; pp < PB; ++pp) {
          qr[pp] = static_cast<double>(sq[i][pp].x);
          qi[pp] = static_cast<double>(sq[i][pp].y);
        }
#pragma unroll
        for (int c = 0; c < K1; ++c) {
          const double w = wxy * sw[i][2][c];
#pragma unroll
          for (int pp = 0; pp < PB; ++pp) {
            ar[c][pp] += w * qr[pp];
            ai[c][pp] += w * qi[pp];
          }
        }
      }
    }
  }
  if (own) {
#pragma unroll
    for (int c = 0; c < K1; ++c)
#pragma unroll
      for (int pp = 0; pp < PB; ++pp)
        if (p0 + pp < P)
          mom[(b * K + t * K1 + c) * P + p0 + pp] = cmake<R>(static_cast<R>(ar[c][pp]), static_cast<R>(ai[c][pp]));
  }
}

// The same moments on FP64 matrix cores for batched planes: per box,
// M[nodes][columns] = W^T[nodes][points] Q[points][columns] (the 2P real
// columns are the interleaved real and imaginary parts of the planes), a
// dense product reduced over the box's points four at a time with 16x16x4
// FP64 MFMA steps.  Node tiles of 16 nodes are dealt to the four wavefronts
// (at most four each, so (qf+1)^3 <= 256); a block covers 32 columns (two
// 16-column tiles: the accumulators stay within two wavefronts per SIMD) and
// all of its box's points, staged through LDS in chunks with their 1D weights.
// Lane l supplies W[point 4 s + l / 16][node l % 16 of the tile] and
// Q[point 4 s + l / 16][column l % 16]; FP64 accumulator element r of lane
// l holds node 4 r + l / 16 and column l % 16.
constexpr int kMomMfmaChunk = 64, kMomMfmaCols = 32;
typedef double mom_d4 __attribute__((ext_vector_type(4)));

template <typename R, int QF>
__global__ void __launch_bounds__(256) k_far_moments_mfma(const int32_t* __restrict__ fbox_start,
                                                          const int32_t* __restrict__ fperm,
                                                          const double* __restrict__ w3, int64_t N,
                                                          const cplx<R>* __restrict__ qint, int P,
                                                          cplx<R>* __restrict__ mom) {
  constexpr int K1 = QF + 1, K = K1 * K1 * K1, NT = (K + 15) / 16, TW = (NT + 3) / 4, CH = kMomMfmaChunk;
  constexpr int NC = kMomMfmaCols, CT = NC / 16;
  static_assert(TW <= 4, "at most four node tiles per wavefront");
  __shared__ double sw[CH][3][K1];
  __shared__ R sq[CH][NC + 1];  // this block's real columns, padded
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int kk = lane >> 4, li = lane & 15;
  const int64_t b = blockIdx.x;
  const int col0 = blockIdx.y * NC;  // first real column of this block
  const int twoP = 2 * P;
  const R* qr = reinterpret_cast<const R*>(qint);
  // this lane's node (A operand row) in each of its tiles
  int na[TW], nb_[TW], nc[TW];
  bool nv[TW];
#pragma unroll
  for (int i = 0; i < TW; ++i) {
    const int k = (wave + 4 * i) * 16 + li;
    nv[i] = (wave + 4 * i) < NT && k < K;
    const int kc = nv[i] ? k : 0;
    na[i] = kc / (K1 * K1);
    nb_[i] = (kc / K1) % K1;
    nc[i] = kc % K1;
  }
  mom_d4 acc[TW][CT];
#pragma unroll
  for (int i = 0; i < TW; ++i)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[i][ct] = mom_d4{0.0, 0.0, 0.0, 0.0};
  const int j0 = fbox_start[b], j1 = fbox_start[b + 1];
  for (int base = j0; base < j1; base += CH) {
    const int cnt = min(CH, j1 - base);
    __syncthreads();
    for (int i = t; i < CH; i += 256) {
      const bool ok = i < cnt;
      const int n = ok ? fperm[base + i] : 0;
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < K1; ++a) sw[i][c][a] = ok ? w3[(c * K1 + a) * N + n] : 0.0;
    }
    for (int e = t; e < CH * NC; e += 256) {
      const int i = e / NC, c = e % NC;
      const bool ok = i < cnt && col0 + c < twoP;
      sq[i][c] = ok ? qr[static_cast<int64_t>(fperm[base + i]) * twoP + col0 + c] : R(0);
    }
    __syncthreads();
    for (int s = 0; s < cnt; s += 4) {
      const int i = s + kk;  // this lane's point (zero weights past cnt)
      double bv[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) bv[ct] = static_cast<double>(sq[i][ct * 16 + li]);
#pragma unroll
      for (int it = 0; it < TW; ++it) {
        if (wave + 4 * it >= NT) break;
        const double av = nv[it] ? sw[i][0][na[it]] * sw[i][1][nb_[it]] * sw[i][2][nc[it]] : 0.0;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
          if (col0 + ct * 16 < twoP) acc[it][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[ct], acc[it][ct], 0, 0, 0);
      }
    }
  }
  R* mr = reinterpret_cast<R*>(mom);
#pragma unroll
  for (int it = 0; it < TW; ++it) {
    if (wave + 4 * it >= NT) break;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int col = col0 + ct * 16 + li;
      if (col >= twoP) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = (wave + 4 * it) * 16 + 4 * r + kk;
        if (k < K) mr[(b * K + k) * twoP + col] = static_cast<R>(acc[it][ct][r]);
      }
    }
  }
}

template <typename R, int QF>
__global__ void k_far_gather(FarArgs f, const cplx<R>* __restrict__ mom, int P, cplx<R>* __restrict__ grid) {
  constexpr int K1 = QF + 1;
  constexpr int K = K1 * K1 * K1;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= f.Ngf * P) return;
  const int64_t g = idx / P;
  const int p = static_cast<int>(idx - g * P);
  const int gz = static_cast<int>(g % f.nf[2]);
  const int gy = static_cast<int>((g / f.nf[2]) % f.nf[1]);
  const int gx = static_cast<int>(g / (static_cast<int64_t>(f.nf[1]) * f.nf[2]));
  double ar = 0.0, ai = 0.0;
  for (int bx = max(0, gx - QF); bx <= min(gx, f.nint[0]); ++bx)
    for (int by = max(0, gy - QF); by <= min(gy, f.nint[1]); ++by)
      for (int bz = max(0, gz - QF); bz <= min(gz, f.nint[2]); ++bz) {
        const int64_t b = (static_cast<int64_t>(bx) * f.nb[1] + by) * f.nb[2] + bz;
        const int k = ((gx - bx) * K1 + (gy - by)) * K1 + (gz - bz);
        cplx<R> v = mom[(b * K + k) * P + p];
        ar += static_cast<double>(v.x);
        ai += static_cast<double>(v.y);
      }
  grid[g * P + p] = cmake<R>(static_cast<R>(ar), static_cast<R>(ai));
}

// part[s][i][p] = sum_{j in split s} K(i, j) in[j][p], with K(i, j) =
// table[base(i) - off(j)] (forward) or conj(table[base(j) - off(i)])
// (conjugate transpose), base(i) = ((ix + nfx - 1) sy + iy + nfy - 1) sz +
// iz + nfz - 1 and off(j) = (jx sy + jy) sz + jz indexing the (2 nf - 1)^3
// offset table.  The splits over j are summed in a fixed order afterwards.
template <typename R, int PB, int BS>
__global__ void __launch_bounds__(BS) k_far_apply(FarArgs f, const cplx<R>* __restrict__ table,
                                                  const cplx<R>* __restrict__ in, cplx<R>* __restrict__ part,
                                                  int P, int adjoint, int64_t jlen) {
  __shared__ cplx<R> sh[PB][BS];
  __shared__ int64_t shi[BS];
  const int64_t sy = 2 * f.nf[1] - 1, sz = 2 * f.nf[2] - 1;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int p0 = blockIdx.y * PB;
  const int split = blockIdx.z;
  const int64_t jbeg = split * jlen, jend = min<int64_t>(f.Ngf, jbeg + jlen);
  const bool active = i < f.Ngf;
  int64_t base_i = 0, off_i = 0;
  if (active) {
    const int iz = static_cast<int>(i % f.nf[2]);
    const int iy = static_cast<int>((i / f.nf[2]) % f.nf[1]);
    const int ix = static_cast<int>(i / (static_cast<int64_t>(f.nf[1]) * f.nf[2]));
    base_i = ((ix + f.nf[0] - 1) * sy + iy + f.nf[1] - 1) * sz + iz + f.nf[2] - 1;
    off_i = (ix * sy + iy) * sz + iz;
  }
  R ar[PB], ai[PB];
#pragma unroll
  for (int pp = 0; pp < PB; ++pp) ar[pp] = ai[pp] = R(0);
  for (int64_t jc = jbeg; jc < jend; jc += BS) {
    const int64_t j = jc + threadIdx.x;
    if (j < jend) {
      const int jz = static_cast<int>(j % f.nf[2]);
      const int jy = static_cast<int>((j / f.nf[2]) % f.nf[1]);
      const int jx = static_cast<int>(j / (static_cast<int64_t>(f.nf[1]) * f.nf[2]));
      shi[threadIdx.x] = adjoint ? ((jx + f.nf[0] - 1) * sy + jy + f.nf[1] - 1) * sz + jz + f.nf[2] - 1
                                 : (jx * sy + jy) * sz + jz;
#pragma unroll
      for (int pp = 0; pp < PB; ++pp)
        sh[pp][threadIdx.x] = (p0 + pp < P) ? in[j * P + p0 + pp] : cmake<R>(R(0), R(0));
    }
    __syncthreads();
    const int cnt = static_cast<int>(min<int64_t>(BS, jend - jc));
    if (active) {
      for (int jj = 0; jj < cnt; ++jj) {
        const int64_t t = adjoint ? (shi[jj] - off_i) : (base_i - shi[jj]);
        cplx<R> kv = table[t];
        if (adjoint) kv.y = -kv.y;
#pragma unroll
        for (int pp = 0; pp < PB; ++pp) {
          const cplx<R> x = sh[pp][jj];
          ar[pp] += kv.x * x.x - kv.y * x.y;
          ai[pp] += kv.x * x.y + kv.y * x.x;
        }
      }
    }
    __syncthreads();
  }
  if (active) {
#pragma unroll
    for (int pp = 0; pp < PB; ++pp)
      if (p0 + pp < P)
        part[(static_cast<int64_t>(split) * f.Ngf + i) * P + p0 + pp] = cmake<R>(ar[pp], ai[pp]);
  }
}

// The same grid sum on the matrix cores once several planes are batched (a
// GEMM, Eq. (8) applied to every right-hand side).  A wavefront owns a 16 x 16
// tile of (grid nodes i) x (planes p) and walks its split of j four at a time
// with 16x16x4 MFMA steps; the K fragment is generated from the offset table
// (lane l supplies K(i0 + l % 16, j + l / 16)), the amplitude fragment is
// in[j + l / 16][p0 + l % 16].  A complex product is four real MFMAs:
// Re += Kr Qr - Ki Qi, Im += Kr Qi + Ki Qr.  Accumulator element r of lane l
// holds column l % 16 and row 4 (l / 16) + r (FP32) or 4 r + l / 16 (FP64);
// both layouts were read off the hardware with one-hot operands.
typedef float mfma_f4 __attribute__((ext_vector_type(4)));
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

template <typename R>
struct MfmaAcc;
template <>
struct MfmaAcc<float> {
  typedef mfma_f4 T;
  static __device__ inline T step(float a, float b, T c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <>
struct MfmaAcc<double> {
  typedef mfma_d4 T;
  static __device__ inline T step(double a, double b, T c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int lane, int r) { return 4 * r + (lane >> 4); }
};

constexpr int kFarMfmaWaves = 4;  // row tiles per block

template <typename R>
__global__ void __launch_bounds__(64 * kFarMfmaWaves) k_far_apply_mfma(FarArgs f, const cplx<R>* __restrict__ table,
                                                                       const cplx<R>* __restrict__ in,
                                                                       cplx<R>* __restrict__ part, int P, int adjoint,
                                                                       int64_t jlen) {
  typedef typename MfmaAcc<R>::T Acc;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t sy = 2 * f.nf[1] - 1, sz = 2 * f.nf[2] - 1;
  const int64_t i0 = (static_cast<int64_t>(blockIdx.x) * kFarMfmaWaves + wave) * 16;
  const int p0 = blockIdx.y * 16;
  const int split = blockIdx.z;
  const int64_t jbeg = split * jlen, jend = min<int64_t>(f.Ngf, jbeg + jlen);
  // this lane's row of the K fragment and column (plane) of the amplitude fragment
  const int64_t ia = i0 + (lane & 15);
  const bool row_ok = ia < f.Ngf;
  const int pb = p0 + (lane & 15);
  const bool col_ok = pb < P;
  const int kk = lane >> 4;
  int64_t base_i = 0, off_i = 0;
  if (row_ok) {
    const int iz = static_cast<int>(ia % f.nf[2]);
    const int iy = static_cast<int>((ia / f.nf[2]) % f.nf[1]);
    const int ix = static_cast<int>(ia / (static_cast<int64_t>(f.nf[1]) * f.nf[2]));
    base_i = ((ix + f.nf[0] - 1) * sy + iy + f.nf[1] - 1) * sz + iz + f.nf[2] - 1;
    off_i = (ix * sy + iy) * sz + iz;
  }
  Acc accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
  for (int64_t jc = jbeg; jc < jend; jc += 4) {
    const int64_t j = jc + kk;
    R kr = R(0), ki = R(0), qr = R(0), qi = R(0);
    if (j < jend) {
      const int jz = static_cast<int>(j % f.nf[2]);
      const int jy = static_cast<int>((j / f.nf[2]) % f.nf[1]);
      const int jx = static_cast<int>(j / (static_cast<int64_t>(f.nf[1]) * f.nf[2]));
      if (row_ok) {
        const int64_t t = adjoint ? (((jx + f.nf[0] - 1) * sy + jy + f.nf[1] - 1) * sz + jz + f.nf[2] - 1) - off_i
                                  : base_i - ((jx * sy + jy) * sz + jz);
        const cplx<R> kv = table[t];
        kr = kv.x;
        ki = adjoint ? -kv.y : kv.y;
      }
      if (col_ok) {
        const cplx<R> qv = in[j * P + pb];
        qr = qv.x;
        qi = qv.y;
      }
    }
    accr = MfmaAcc<R>::step(kr, qr, accr);
    accr = MfmaAcc<R>::step(-ki, qi, accr);
    acci = MfmaAcc<R>::step(kr, qi, acci);
    acci = MfmaAcc<R>::step(ki, qr, acci);
  }
  const int pc = p0 + (lane & 15);
  if (pc < P) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t io = i0 + MfmaAcc<R>::row(lane, r);
      if (io < f.Ngf)
        part[(static_cast<int64_t>(split) * f.Ngf + io) * P + pc] = cmake<R>(accr[r], acci[r]);
    }
  }
}

// The same GEMM with bfloat16 inputs and FP32 accumulation (16x16x16 bf16
// MFMA, four k per lane): lane l supplies K(i0 + l % 16, j + 4 (l / 16) + v)
// and in[j + 4 (l / 16) + v][p0 + l % 16] for v = 0..3; the accumulator layout
// is the FP32 one above.  Both were checked on the hardware against a host
// product of small integers.  Inputs are rounded to nearest even on the upper
// half of their binary32 encoding (the bfloat16 format).  X3: each input is
// split as hi + lo (hi = bf16(x), lo = bf16(x - hi)) and a product is taken
// as lo·hi + hi·lo + hi·hi (the three-term bfloat16 splitting of Henry, Tang
// and Heinecke, 2019), which recovers about 16 significant bits.
typedef short bf16x4 __attribute__((ext_vector_type(4)));

__device__ inline short bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<short>(u >> 16);
}

__device__ inline float bf16_value(short h) {
  return __uint_as_float(static_cast<uint32_t>(static_cast<uint16_t>(h)) << 16);
}

// x = hi + lo to about 16 significant bits
__device__ inline void bf16_split(float x, short& hi, short& lo) {
  hi = bf16_rne(x);
  lo = bf16_rne(x - bf16_value(hi));
}

__device__ inline mfma_f4 mfma_bf16(bf16x4 a, bf16x4 b, mfma_f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

template <bool X3>
__global__ void __launch_bounds__(64 * kFarMfmaWaves) k_far_apply_mfma_bf16(FarArgs f,
                                                                            const cplx<float>* __restrict__ table,
                                                                            const cplx<float>* __restrict__ in,
                                                                            cplx<float>* __restrict__ part, int P,
                                                                            int adjoint, int64_t jlen) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t sy = 2 * f.nf[1] - 1, sz = 2 * f.nf[2] - 1;
  const int64_t i0 = (static_cast<int64_t>(blockIdx.x) * kFarMfmaWaves + wave) * 16;
  const int p0 = blockIdx.y * 16;
  const int split = blockIdx.z;
  const int64_t jbeg = split * jlen, jend = min<int64_t>(f.Ngf, jbeg + jlen);
  const int64_t ia = i0 + (lane & 15);
  const bool row_ok = ia < f.Ngf;
  const int pb = p0 + (lane & 15);
  const bool col_ok = pb < P;
  const int kg = lane >> 4;
  int64_t base_i = 0, off_i = 0;
  if (row_ok) {
    const int iz = static_cast<int>(ia % f.nf[2]);
    const int iy = static_cast<int>((ia / f.nf[2]) % f.nf[1]);
    const int ix = static_cast<int>(ia / (static_cast<int64_t>(f.nf[1]) * f.nf[2]));
    base_i = ((ix + f.nf[0] - 1) * sy + iy + f.nf[1] - 1) * sz + iz + f.nf[2] - 1;
    off_i = (ix * sy + iy) * sz + iz;
  }
  mfma_f4 accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
  for (int64_t jc = jbeg; jc < jend; jc += 16) {
    bf16x4 kr, kin, ki, qr, qi;     // hi parts (the only parts without X3)
    bf16x4 krl, kinl, kil, qrl, qil;  // lo parts
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t j = jc + 4 * kg + v;
      float a = 0.f, b = 0.f, c = 0.f, d = 0.f;
      if (j < jend) {
        const int jz = static_cast<int>(j % f.nf[2]);
        const int jy = static_cast<int>((j / f.nf[2]) % f.nf[1]);
        const int jx = static_cast<int>(j / (static_cast<int64_t>(f.nf[1]) * f.nf[2]));
        if (row_ok) {
          const int64_t t = adjoint ? (((jx + f.nf[0] - 1) * sy + jy + f.nf[1] - 1) * sz + jz + f.nf[2] - 1) - off_i
                                    : base_i - ((jx * sy + jy) * sz + jz);
          const cplx<float> kv = table[t];
          a = kv.x;
          b = adjoint ? -kv.y : kv.y;
        }
        if (col_ok) {
          const cplx<float> qv = in[j * P + pb];
          c = qv.x;
          d = qv.y;
        }
      }
      if (X3) {
        short h, l;
        bf16_split(a, h, l);
        kr[v] = h;
        krl[v] = l;
        bf16_split(b, h, l);
        ki[v] = h;
        kil[v] = l;
        bf16_split(-b, h, l);
        kin[v] = h;
        kinl[v] = l;
        bf16_split(c, h, l);
        qr[v] = h;
        qrl[v] = l;
        bf16_split(d, h, l);
        qi[v] = h;
        qil[v] = l;
      } else {
        kr[v] = bf16_rne(a);
        ki[v] = bf16_rne(b);
        kin[v] = bf16_rne(-b);
        qr[v] = bf16_rne(c);
        qi[v] = bf16_rne(d);
      }
    }
    if (X3) {
      accr = mfma_bf16(krl, qr, accr);
      accr = mfma_bf16(kr, qrl, accr);
      accr = mfma_bf16(kinl, qi, accr);
      accr = mfma_bf16(kin, qil, accr);
      acci = mfma_bf16(krl, qi, acci);
      acci = mfma_bf16(kr, qil, acci);
      acci = mfma_bf16(kil, qr, acci);
      acci = mfma_bf16(ki, qrl, acci);
    }
    accr = mfma_bf16(kr, qr, accr);
    accr = mfma_bf16(kin, qi, accr);
    acci = mfma_bf16(kr, qi, acci);
    acci = mfma_bf16(ki, qr, acci);
  }
  const int pc = p0 + (lane & 15);
  if (pc < P) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t io = i0 + 4 * (lane >> 4) + r;
      if (io < f.Ngf) part[(static_cast<int64_t>(split) * f.Ngf + io) * P + pc] = cmake<float>(accr[r], acci[r]);
    }
  }
}

// Step 3 with batched planes.  All points of a far box share one stencil
// (the boxes are keyed by the stencil start), so a block stages the box's
// (qf+1)^3 nodes x P planes in LDS once and interpolates a chunk of the box's
// points from there, lanes over planes (LP planes x 64 / LP points per
// wavefront).
constexpr int kFarInterpChunk = 256;

template <typename R, int QF, int LP>
__global__ void __launch_bounds__(256) k_far_interp_box(FarArgs f, const int32_t* __restrict__ fbox_start,
                                                        const int32_t* __restrict__ fperm,
                                                        const int32_t* __restrict__ s3, const double* __restrict__ w3,
                                                        int64_t N, const cplx<R>* __restrict__ grid, int P,
                                                        cplx<R>* __restrict__ u, int accumulate) {
  extern __shared__ unsigned char lds_raw[];
  cplx<R>* sg = reinterpret_cast<cplx<R>*>(lds_raw);  // [K][P]
  constexpr int K1 = QF + 1;
  constexpr int K = K1 * K1 * K1;
  constexpr int E = 64 / LP;
  const int64_t b = blockIdx.x;
  const int jb = fbox_start[b] + blockIdx.y * kFarInterpChunk;
  const int je = min(fbox_start[b + 1], jb + kFarInterpChunk);
  if (jb >= je) return;  // the whole block leaves together
  const int m0 = fperm[fbox_start[b]];
  const int sx = s3[m0], sy = s3[N + m0], sz = s3[2 * N + m0];
  for (int t = threadIdx.x; t < K * P; t += blockDim.x) {
    const int k = t / P, p = t - k * P;
    const int a = k / (K1 * K1), bb = (k / K1) % K1, c = k % K1;
    const int64_t node = (static_cast<int64_t>(sx + a) * f.nf[1] + (sy + bb)) * f.nf[2] + (sz + c);
    sg[t] = grid[node * P + p];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int e = lane / LP, pl = lane % LP;
  const int slot = (threadIdx.x >> 6) * E + e;
  for (int j = jb + slot; j < je; j += (blockDim.x >> 6) * E) {
    const int m = fperm[j];
    double wx[K1], wy[K1], wz[K1];
#pragma unroll
    for (int a = 0; a < K1; ++a) {
      wx[a] = w3[a * N + m];
      wy[a] = w3[(K1 + a) * N + m];
      wz[a] = w3[(2 * K1 + a) * N + m];
    }
    for (int pc = 0; pc < P; pc += LP) {
      const int p = pc + pl;
      if (p >= P) continue;
      double ar = 0.0, ai = 0.0;
      for (int a = 0; a < K1; ++a)
        for (int bb = 0; bb < K1; ++bb) {
          const double wab = wx[a] * wy[bb];
          const cplx<R>* row = sg + ((a * K1 + bb) * K1) * P + p;
#pragma unroll
          for (int c = 0; c < K1; ++c) {
            const cplx<R> v = row[c * P];
            const double w = wab * wz[c];
            ar += w * static_cast<double>(v.x);
            ai += w * static_cast<double>(v.y);
          }
        }
      cplx<R>* o = u + static_cast<int64_t>(m) * P + p;
      cplx<R> r = cmake<R>(static_cast<R>(ar), static_cast<R>(ai));
      if (accumulate) r = cadd(*o, r);
      *o = r;
    }
  }
}

// The same interpolation on FP64 matrix cores.  With W[m][(a, b, c)] =
// wx_m[a] wy_m[b] wz_m[c] shared by all points of the box, it is the dense
// product U[points][columns] = W[points][nodes] G[nodes][columns], the 2P
// real columns being the interleaved real and imaginary parts of the planes
// (W is real).  A wavefront owns RT 16-point row tiles and CT 16-column
// tiles and walks the (qf+1)^3 nodes four at a time in their linear order
// (a, b, c) (one 16x16x4 step each, the last one padded with zero weights).
// Lane l supplies W[point l % 16][node 4 s + l / 16] and G[that node][column
// l % 16]; accumulation is FP64, as in the vector form above.
constexpr int kFimRT = 2, kFimCT = 4;
constexpr int kFimPts = 4 * 16 * kFimRT;  // points per block

template <typename R, int QF>
__global__ void __launch_bounds__(256) k_far_interp_mfma(FarArgs f, const int32_t* __restrict__ fbox_start,
                                                         const int32_t* __restrict__ fperm,
                                                         const int32_t* __restrict__ s3, const double* __restrict__ w3,
                                                         int64_t N, const cplx<R>* __restrict__ grid, int P,
                                                         cplx<R>* __restrict__ u, int accumulate) {
  constexpr int K1 = QF + 1, K = K1 * K1 * K1, NS = (K + 3) / 4;
  constexpr int RT = kFimRT, CT = kFimCT;
  extern __shared__ unsigned char lds_raw[];
  double* sw = reinterpret_cast<double*>(lds_raw);           // [kFimPts][3][K1]
  int* sperm = reinterpret_cast<int*>(sw + kFimPts * 3 * K1);  // [kFimPts]
  cplx<R>* sg = reinterpret_cast<cplx<R>*>(sperm + kFimPts);  // [K][P]
  const int64_t b = blockIdx.x;
  const int jb = fbox_start[b] + blockIdx.y * kFimPts;
  const int je = min(fbox_start[b + 1], jb + kFimPts);
  if (jb >= je) return;  // the whole block leaves together
  const int np = je - jb;
  const int m0 = fperm[fbox_start[b]];
  const int sx = s3[m0], sy = s3[N + m0], sz = s3[2 * N + m0];
  for (int t = threadIdx.x; t < K * P; t += blockDim.x) {
    const int k = t / P, p = t - k * P;
    const int a = k / (K1 * K1), bb = (k / K1) % K1, c = k % K1;
    const int64_t node = (static_cast<int64_t>(sx + a) * f.nf[1] + (sy + bb)) * f.nf[2] + (sz + c);
    sg[t] = grid[node * P + p];
  }
  for (int t = threadIdx.x; t < np; t += blockDim.x) {
    const int m = fperm[jb + t];
    sperm[t] = m;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < K1; ++a) sw[(t * 3 + c) * K1 + a] = w3[(c * K1 + a) * N + m];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kk = lane >> 4, li = lane & 15;
  const int twoP = 2 * P;
  const R* sgr = reinterpret_cast<const R*>(sg);
  // this lane's point in each row tile (A operand)
  int pt[RT];
  bool pv[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    pt[rt] = (wave * RT + rt) * 16 + li;
    pv[rt] = pt[rt] < np;
    if (!pv[rt]) pt[rt] = 0;  // its weights are replaced by zero below
  }
  for (int pc = 0; pc < twoP; pc += 16 * CT) {
    mfma_d4 acc[RT][CT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = mfma_d4{0.0, 0.0, 0.0, 0.0};
    for (int st = 0; st < NS; ++st) {
      const int node = 4 * st + kk;
      const bool nv = node < K;
      const int nd = nv ? node : 0;
      const int a = nd / (K1 * K1), bb = (nd / K1) % K1, c = nd % K1;
      double bv[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int col = pc + ct * 16 + li;
        bv[ct] = (nv && col < twoP) ? static_cast<double>(sgr[nd * twoP + col]) : 0.0;
      }
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const double* w = sw + pt[rt] * 3 * K1;
        const double av = (nv && pv[rt]) ? w[a] * w[K1 + bb] * w[2 * K1 + c] : 0.0;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
          if (pc + ct * 16 < twoP) acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[ct], acc[rt][ct], 0, 0, 0);
      }
    }
    // element r of lane l: row 4 r + l / 16, column l % 16
    R* ur = reinterpret_cast<R*>(u);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int col = pc + ct * 16 + li;
        if (col >= twoP) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = (wave * RT + rt) * 16 + 4 * r + kk;
          if (row < np) {
            R* o = ur + static_cast<int64_t>(sperm[row]) * twoP + col;
            const R v = static_cast<R>(acc[rt][ct][r]);
            *o = accumulate ? *o + v : v;
          }
        }
      }
  }
}

template <typename R, int QF>
static bool far_interp_box_q(const FarArgs& f, const int32_t* fbox_start, const int32_t* fperm, int max_box,
                             const int32_t* s3, const double* w3, int64_t N, const void* grid, int P, void* u,
                             bool acc, hipStream_t st) {
  constexpr int K = (QF + 1) * (QF + 1) * (QF + 1);
  const size_t lds = static_cast<size_t>(K) * P * sizeof(cplx<R>);
  if (P < 8) return false;
  const size_t lds_m = lds + static_cast<size_t>(kFimPts) * (3 * (QF + 1) * sizeof(double) + sizeof(int));
  if (lds_m <= 128 * 1024) {
    dim3 gm(static_cast<unsigned>(f.nboxes), static_cast<unsigned>((max_box + kFimPts - 1) / kFimPts));
    hipLaunchKernelGGL((k_far_interp_mfma<R, QF>), gm, dim3(256), lds_m, st, f, fbox_start, fperm, s3, w3, N,
                       static_cast<const cplx<R>*>(grid), P, static_cast<cplx<R>*>(u), acc ? 1 : 0);
    return true;
  }
  if (lds > 128 * 1024) return false;
  dim3 gr(static_cast<unsigned>(f.nboxes), static_cast<unsigned>((max_box + kFarInterpChunk - 1) / kFarInterpChunk));
#define FFTPIM_FIB(LPV)                                                                                    \
  hipLaunchKernelGGL((k_far_interp_box<R, QF, LPV>), gr, dim3(256), lds, st, f, fbox_start, fperm, s3, w3, N, \
                     static_cast<const cplx<R>*>(grid), P, static_cast<cplx<R>*>(u), acc ? 1 : 0)
  if (P <= 16)
    FFTPIM_FIB(16);
  else if (P <= 32)
    FFTPIM_FIB(32);
  else
    FFTPIM_FIB(64);
#undef FFTPIM_FIB
  return true;
}

template <typename R>
bool launch_far_interp_box(int qf, const FarArgs& f, const int32_t* fbox_start, const int32_t* fperm, int max_box,
                           const int32_t* s3, const double* w3, int64_t N, const void* grid, int P, void* u, bool acc,
                           hipStream_t st) {
  if (max_box <= 0) return false;
  switch (qf) {
    case 1: return far_interp_box_q<R, 1>(f, fbox_start, fperm, max_box, s3, w3, N, grid, P, u, acc, st);
    case 2: return far_interp_box_q<R, 2>(f, fbox_start, fperm, max_box, s3, w3, N, grid, P, u, acc, st);
    case 3: return far_interp_box_q<R, 3>(f, fbox_start, fperm, max_box, s3, w3, N, grid, P, u, acc, st);
    case 4: return far_interp_box_q<R, 4>(f, fbox_start, fperm, max_box, s3, w3, N, grid, P, u, acc, st);
    case 5: return far_interp_box_q<R, 5>(f, fbox_start, fperm, max_box, s3, w3, N, grid, P, u, acc, st);
    case 6: return far_interp_box_q<R, 6>(f, fbox_start, fperm, max_box, s3, w3, N, grid, P, u, acc, st);
    case 7: return far_interp_box_q<R, 7>(f, fbox_start, fperm, max_box, s3, w3, N, grid, P, u, acc, st);
    default: return false;
  }
}

template <typename R>
__global__ void k_far_reduce(const cplx<R>* __restrict__ part, cplx<R>* __restrict__ out, int64_t n, int nsplit) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  cplx<R> s = part[idx];
  for (int k = 1; k < nsplit; ++k) s = cadd(s, part[static_cast<int64_t>(k) * n + idx]);
  out[idx] = s;
}

// ---------------------------------------------------------------------------
// plan time: the far-zone table for 2D-periodic kernels with k0 or a phase
// shift, on the device.  Entry e is G^p(r) - sum_{|i| <= i_d} phase_i G0(r -
// R_i) at the offset r of the shifted observer and source grids (Sec. 3.2),
// G^p from the Floquet series of Eq. (pgf_2) after reducing r into the cell
// (Bloch phase).  One block per entry; threads take Floquet orders m, loop
// over n, and the partial sums are added in a fixed tree order.
// ---------------------------------------------------------------------------

constexpr int kTableThreads = 256;

// CW: complex wavenumbers (a lossy k0 or a complex phase shift); the real
// instantiation keeps the propagating / evanescent split in real arithmetic.
template <bool CW>
__global__ void __launch_bounds__(kTableThreads) k_far_table_pgf2(FarTableArgs a, cplx<double>* __restrict__ table) {
  __shared__ double shr[kTableThreads], shi[kTableThreads];
  const double pi = 3.14159265358979323846;
  const int sy = 2 * a.nf[1] - 1, sz = 2 * a.nf[2] - 1;
  const int64_t e = blockIdx.x;
  const int dz = static_cast<int>(e % sz), dy = static_cast<int>((e / sz) % sy),
            dx = static_cast<int>(e / (static_cast<int64_t>(sz) * sy));
  const double r0[3] = {(dx - (a.nf[0] - 1) - 0.5) * a.delta[0], (dy - (a.nf[1] - 1) - 0.5) * a.delta[1],
                        (dz - (a.nf[2] - 1) - 0.5) * a.delta[2]};
  const cplx<double> k0 = cmake<double>(a.k0, a.k0_im);
  const cplx<double> kt0 = cmake<double>(a.kt[0], a.kt_im[0]), kt1 = cmake<double>(a.kt[1], a.kt_im[1]);
  // reduce x, y into the cell; Bloch phase of the shift, exp(-j arg)
  double r[3] = {r0[0], r0[1], r0[2]};
  cplx<double> arg = cmake<double>(0.0, 0.0);
  for (int c = 0; c < 2; ++c) {
    const double n = round(r[c] / a.L[c]);
    r[c] -= n * a.L[c];
    arg = cadd(arg, cscale(c == 0 ? kt0 : kt1, n * a.L[c]));
  }
  const double az = fabs(r[2]);
  const double kreach = 41.0 / az + hypot(a.k0, a.k0_im) + hypot(a.kt[0], a.kt_im[0]) + hypot(a.kt[1], a.kt_im[1]);
  const int mmax = static_cast<int>(ceil(kreach * a.L[0] / (2.0 * pi))) + 1;
  const int nmax = static_cast<int>(ceil(kreach * a.L[1] / (2.0 * pi))) + 1;
  double sr = 0.0, si = 0.0;
  for (int m = -mmax + static_cast<int>(threadIdx.x); m <= mmax; m += kTableThreads) {
    if (CW) {
      const cplx<double> kx = cadd(kt0, cmake<double>(2.0 * pi * m / a.L[0], 0.0));
      const cplx<double> kx2 = cmul(kx, kx);
      cplx<double> part = cmake<double>(0.0, 0.0);
      for (int n = -nmax; n <= nmax; ++n) {
        const cplx<double> ky = cadd(kt1, cmake<double>(2.0 * pi * n / a.L[1], 0.0));
        const cplx<double> w = csub(csub(cmul(k0, k0), kx2), cmul(ky, ky));
        const cplx<double> kz = csqrt_im_nonpos_d(w);
        // exp(-j (ky y + kz |z|)) / kz
        const cplx<double> ex = cadd(cscale(ky, r[1]), cscale(kz, az));
        part = cadd(part, cdiv_d(cexp_d(cmake<double>(ex.y, -ex.x)), kz));
      }
      const cplx<double> exx = cexp_d(cmake<double>(kx.y * r[0], -kx.x * r[0]));
      const cplx<double> t = cmul(exx, part);
      sr += t.x;
      si += t.y;
    } else {
      const double kx = a.kt[0] + 2.0 * pi * m / a.L[0];
      double pr = 0.0, pim = 0.0;
      for (int n = -nmax; n <= nmax; ++n) {
        const double ky = a.kt[1] + 2.0 * pi * n / a.L[1];
        const double w = a.k0 * a.k0 - kx * kx - ky * ky;
        double s, c;
        if (w >= 0.0) {
          // propagating: exp(-j (ky y + kz |z|)) / kz
          const double kz = sqrt(w);
          sincos(-(ky * r[1] + kz * az), &s, &c);
          pr += c / kz;
          pim += s / kz;
        } else {
          // evanescent, kz = -j kappa: j exp(-kappa |z|) exp(-j ky y) / kappa
          const double kap = sqrt(-w);
          sincos(-ky * r[1], &s, &c);
          const double fct = exp(-kap * az) / kap;
          pr -= s * fct;
          pim += c * fct;
        }
      }
      double s, c;
      sincos(-kx * r[0], &s, &c);
      sr += c * pr - s * pim;
      si += c * pim + s * pr;
    }
  }
  shr[threadIdx.x] = sr;
  shi[threadIdx.x] = si;
  __syncthreads();
  for (int h = kTableThreads / 2; h > 0; h >>= 1) {
    if (static_cast<int>(threadIdx.x) < h) {
      shr[threadIdx.x] += shr[threadIdx.x + h];
      shi[threadIdx.x] += shi[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  // divide by 2 j Lx Ly, apply the Bloch phase exp(-j arg)
  const double inv = 1.0 / (2.0 * a.L[0] * a.L[1]);
  const cplx<double> g = cmake<double>(shi[0] * inv, -shr[0] * inv);
  cplx<double> out = cmul(cexp_d(cmake<double>(arg.y, -arg.x)), g);
  // minus the near-zone images (unreduced offset)
  for (int ix = -a.id; ix <= a.id; ++ix)
    for (int iy = -a.id; iy <= a.id; ++iy) {
      const double Rx = ix * a.L[0], Ry = iy * a.L[1];
      const double ddx = r0[0] - Rx, ddy = r0[1] - Ry, ddz = r0[2];
      const double dist = sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
      // phase exp(-j (kt . R)) times exp(-j k0 dist) / (4 pi dist)
      const cplx<double> ph = cadd(cadd(cscale(kt0, Rx), cscale(kt1, Ry)), cscale(k0, dist));
      out = csub(out, cscale(cexp_d(cmake<double>(ph.y, -ph.x)), 1.0 / (4.0 * pi * dist)));
    }
  table[e] = out;
}

void launch_far_table_pgf2(const FarTableArgs& a, void* table, hipStream_t st) {
  const int64_t total = static_cast<int64_t>(2 * a.nf[0] - 1) * (2 * a.nf[1] - 1) * (2 * a.nf[2] - 1);
  const bool cw = a.k0_im != 0.0 || a.kt_im[0] != 0.0 || a.kt_im[1] != 0.0;
  if (cw)
    hipLaunchKernelGGL(k_far_table_pgf2<true>, dim3(static_cast<unsigned>(total)), dim3(kTableThreads), 0, st, a,
                       static_cast<cplx<double>*>(table));
  else
    hipLaunchKernelGGL(k_far_table_pgf2<false>, dim3(static_cast<unsigned>(total)), dim3(kTableThreads), 0, st, a,
                       static_cast<cplx<double>*>(table));
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <typename R, int QF>
static void moments_q(const FarArgs& f, const int32_t* fbox_start, const int32_t* fperm, const double* u3,
                      int64_t N, const void* qint, int P, void* mom, hipStream_t st) {
  constexpr int K1 = QF + 1;
  const int bs = ((K1 * K1 + 63) / 64) * 64;
#define FFTPIM_MOM(PBV)                                                                                     \
  do {                                                                                                      \
    dim3 gr(static_cast<unsigned>(f.nboxes), (P + PBV - 1) / PBV);                                          \
    hipLaunchKernelGGL((k_far_moments<R, QF, PBV>), gr, dim3(bs), 0, st, fbox_start, fperm, u3, N,          \
                       static_cast<const cplx<R>*>(qint), P, static_cast<cplx<R>*>(mom));                   \
  } while (0)
  if constexpr (K1 <= 6) {
    if (P >= 8) {
      // batched planes: the matrix-core form
      dim3 gm(static_cast<unsigned>(f.nboxes), (2 * P + kMomMfmaCols - 1) / kMomMfmaCols);
      hipLaunchKernelGGL((k_far_moments_mfma<R, QF>), gm, dim3(256), 0, st, fbox_start, fperm, u3, N,
                         static_cast<const cplx<R>*>(qint), P, static_cast<cplx<R>*>(mom));
      return;
    }
  }
  // accumulators: (qf+1) z nodes x PB planes per thread
  if (P >= 4 && K1 <= 6)
    FFTPIM_MOM(4);
  else if (P >= 2)
    FFTPIM_MOM(2);
  else
    FFTPIM_MOM(1);
#undef FFTPIM_MOM
}

template <typename R>
int launch_far_moments(int qf, const FarArgs& f, const int32_t* fbox_start, const int32_t* fperm,
                       const double* u3, int64_t N, const void* qint, int P, void* mom, hipStream_t st) {
  switch (qf) {
    case 1: moments_q<R, 1>(f, fbox_start, fperm, u3, N, qint, P, mom, st); break;
    case 2: moments_q<R, 2>(f, fbox_start, fperm, u3, N, qint, P, mom, st); break;
    case 3: moments_q<R, 3>(f, fbox_start, fperm, u3, N, qint, P, mom, st); break;
    case 4: moments_q<R, 4>(f, fbox_start, fperm, u3, N, qint, P, mom, st); break;
    case 5: moments_q<R, 5>(f, fbox_start, fperm, u3, N, qint, P, mom, st); break;
    case 6: moments_q<R, 6>(f, fbox_start, fperm, u3, N, qint, P, mom, st); break;
    case 7: moments_q<R, 7>(f, fbox_start, fperm, u3, N, qint, P, mom, st); break;
    case 8: moments_q<R, 8>(f, fbox_start, fperm, u3, N, qint, P, mom, st); break;
    case 9: moments_q<R, 9>(f, fbox_start, fperm, u3, N, qint, P, mom, st); break;
    default: return FFTPIM_ERR_UNSUPPORTED;
  }
  return FFTPIM_OK;
}

template <typename R, int QF>
static void gather_q(const FarArgs& f, const void* mom, int P, void* grid, hipStream_t st) {
  const int64_t total = f.Ngf * P;
  hipLaunchKernelGGL((k_far_gather<R, QF>), dim3(static_cast<unsigned>((total + kFarBlock - 1) / kFarBlock)),
                     dim3(kFarBlock), 0, st, f, static_cast<const cplx<R>*>(mom), P, static_cast<cplx<R>*>(grid));
}

template <typename R>
int launch_far_gather(int qf, const FarArgs& f, const void* mom, int P, void* grid, hipStream_t st) {
  switch (qf) {
    case 1: gather_q<R, 1>(f, mom, P, grid, st); break;
    case 2: gather_q<R, 2>(f, mom, P, grid, st); break;
    case 3: gather_q<R, 3>(f, mom, P, grid, st); break;
    case 4: gather_q<R, 4>(f, mom, P, grid, st); break;
    case 5: gather_q<R, 5>(f, mom, P, grid, st); break;
    case 6: gather_q<R, 6>(f, mom, P, grid, st); break;
    case 7: gather_q<R, 7>(f, mom, P, grid, st); break;
    case 8: gather_q<R, 8>(f, mom, P, grid, st); break;
    case 9: gather_q<R, 9>(f, mom, P, grid, st); break;
    default: return FFTPIM_ERR_UNSUPPORTED;
  }
  return FFTPIM_OK;
}

int far_apply_splits(int64_t Ngf, int P) {
  const int64_t blocks = ((Ngf + kFarBlock - 1) / kFarBlock) * ((P + 3) / 4);
  int s = static_cast<int>(std::min<int64_t>(64, std::max<int64_t>(1, (8192 + blocks - 1) / blocks)));
  return static_cast<int>(std::min<int64_t>(s, std::max<int64_t>(1, (Ngf + 255) / 256)));
}

// Planes at or above which the grid sum runs on the matrix cores.
constexpr int kFarMfmaMinPlanes = 8;

template <typename R>
void launch_far_apply(const FarArgs& f, const void* table, const void* in, void* out, void* part, int P,
                      bool adjoint, int bf16_in, hipStream_t st) {
  if (P >= kFarMfmaMinPlanes) {
    // bfloat16 inputs step j 16 at a time
    const int64_t kstep = (bf16_in != 0 && sizeof(R) == 4) ? 16 : 4;
    // split j so the launch has a few blocks per compute unit, within the
    // part buffer's split capacity
    const int64_t row_blocks = (f.Ngf + 16 * kFarMfmaWaves - 1) / (16 * kFarMfmaWaves);
    const int64_t col_blocks = (P + 15) / 16;
    int64_t ns = std::max<int64_t>(1, 1024 / std::max<int64_t>(1, row_blocks * col_blocks));
    ns = std::min<int64_t>(ns, std::min<int64_t>(64, std::max<int64_t>(1, (f.Ngf + 255) / 256)));
    const int64_t jlen = (((f.Ngf + ns - 1) / ns + kstep - 1) / kstep) * kstep;
    const int nsplit = static_cast<int>((f.Ngf + jlen - 1) / jlen);
    dim3 gr(static_cast<unsigned>(row_blocks), static_cast<unsigned>(col_blocks), static_cast<unsigned>(nsplit));
    if (kstep == 16 && bf16_in == 2)
      hipLaunchKernelGGL(k_far_apply_mfma_bf16<true>, gr, dim3(64 * kFarMfmaWaves), 0, st, f,
                         static_cast<const cplx<float>*>(table), static_cast<const cplx<float>*>(in),
                         static_cast<cplx<float>*>(part), P, adjoint ? 1 : 0, jlen);
    else if (kstep == 16)
      hipLaunchKernelGGL(k_far_apply_mfma_bf16<false>, gr, dim3(64 * kFarMfmaWaves), 0, st, f,
                         static_cast<const cplx<float>*>(table), static_cast<const cplx<float>*>(in),
                         static_cast<cplx<float>*>(part), P, adjoint ? 1 : 0, jlen);
    else
      hipLaunchKernelGGL((k_far_apply_mfma<R>), gr, dim3(64 * kFarMfmaWaves), 0, st, f,
                         static_cast<const cplx<R>*>(table), static_cast<const cplx<R>*>(in),
                         static_cast<cplx<R>*>(part), P, adjoint ? 1 : 0, jlen);
    const int64_t n = f.Ngf * P;
    hipLaunchKernelGGL((k_far_reduce<R>), dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st,
                       static_cast<const cplx<R>*>(part), static_cast<cplx<R>*>(out), n, nsplit);
    return;
  }
  const unsigned nb = static_cast<unsigned>((f.Ngf + kFarBlock - 1) / kFarBlock);
  const int ns = far_apply_splits(f.Ngf, P);
  const int64_t jlen = (((f.Ngf + ns - 1) / ns + kFarBlock - 1) / kFarBlock) * kFarBlock;
  const int nsplit = static_cast<int>((f.Ngf + jlen - 1) / jlen);
#define FFTPIM_FARAPPLY(PBV)                                                                               \
  do {                                                                                                     \
    dim3 gr(nb, (P + PBV - 1) / PBV, nsplit);                                                              \
    hipLaunchKernelGGL((k_far_apply<R, PBV, kFarBlock>), gr, dim3(kFarBlock), 0, st, f,                   \
                       static_cast<const cplx<R>*>(table),                                                 \
                       static_cast<const cplx<R>*>(in), static_cast<cplx<R>*>(part), P, adjoint ? 1 : 0,   \
                       jlen);                                                                              \
  } while (0)
  if (P >= 4)
    FFTPIM_FARAPPLY(4);
  else if (P >= 2)
    FFTPIM_FARAPPLY(2);
  else
    FFTPIM_FARAPPLY(1);
#undef FFTPIM_FARAPPLY
  const int64_t n = f.Ngf * P;
  hipLaunchKernelGGL((k_far_reduce<R>), dim3(static_cast<unsigned>((n + kFarBlock - 1) / kFarBlock)), dim3(kFarBlock),
                     0, st, static_cast<const cplx<R>*>(part), static_cast<cplx<R>*>(out), n, nsplit);
}

#define FFTPIM_INST_FAR(R)                                                                                 \
  template int launch_far_moments<R>(int, const FarArgs&, const int32_t*, const int32_t*, const double*,   \
                                     int64_t, const void*, int, void*, hipStream_t);                       \
  template int launch_far_gather<R>(int, const FarArgs&, const void*, int, void*, hipStream_t);            \
  template void launch_far_apply<R>(const FarArgs&, const void*, const void*, void*, void*, int, bool, int,    \
                                    hipStream_t);                                                          \
  template bool launch_far_interp_box<R>(int, const FarArgs&, const int32_t*, const int32_t*, int, const int32_t*, \
                                         const double*, int64_t, const void*, int, void*, bool, hipStream_t);

FFTPIM_INST_FAR(double)
FFTPIM_INST_FAR(float)

}  // namespace fftpim
