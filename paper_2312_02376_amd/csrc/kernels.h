// Kernel argument structs and launcher declarations shared by the kernel
// translation units and the plan/apply orchestration.
#pragma once

#include "common.h"

namespace fftpim {

// Per-point interpolation data used by the kernels: stencil starts s3[c][N]
// and the 1D Lagrange weights w3[c][a][N] (a = 0..q), both in plan order.

// Geometry of one grid as the kernels see it.
struct GridArgs {
  int n[3];     // nodes per axis
  int nint[3];  // cells per axis (box index range 0..nint)
  int nb[3];    // boxes per axis (nint + 1)
};

// One batched 1D FFT pass.  The data is viewed as outer x line x column; the
// transform runs along the line.  contig = 1: lines are contiguous (in_line
// = 1) and a block takes T consecutive outer indices; contig = 0: a block takes
// one outer index and T consecutive columns (coalesced across the block; the
// last tile of a row of columns may be partial).  Grids keep the planes
// innermost ([x][y][z][P]), so for batched planes every node is one
// contiguous run of P values.
struct FftPassDesc {
  int M, logM;         // transform length (power of 2)
  int n_in, n_out;     // nonzero inputs / outputs kept along the line
  int T;               // lines per block
  int contig;
  int64_t ncols, nouter;
  int64_t in_line, in_col, in_outer;
  int64_t out_line, out_col, out_outer;
  int64_t spec_line, spec_col;  // spectrum strides (fused pass only) ...
  int64_t spec_div;             // ... applied to column / spec_div (planes share a spectrum)
};

struct NearTableArgs {
  int M[3], n[3], nint[3];
  double h[3];
  double k0, k0_im;
  int nimg;
  const int* img;        // device [nimg][3] image offsets
  const double* phase;   // device [nimg][2] image phases
};

// In-cell correction stored once per unordered pair of non-empty near-grid
// boxes ("ebox" = index into the list of non-empty boxes); see SymGroup.
struct SymArgs {
  int64_t N;
  int nb[3];
  int R, W;             // g0 table geometry (as in CorrArgs)
  double k0, k0_im;
  int max_box;          // largest point count of a box
  int64_t npairs, nitems, nebox;
  const int32_t* box_start;      // [nb^3 + 1]
  const int32_t* ebox;           // [E] box id of each non-empty box
  const int32_t* pair_ebox_o;    // [npairs] observer-side box (B)     (plan-time fill)
  const int32_t* pair_ebox_s;    // [npairs] source-side box (B' >= B)
  const int64_t* pair_voff;      // [npairs] value of row 0, column 0 of the block
  const int64_t* pair_stride;    // [npairs] row stride
  const SymGroup* groups;        // lane groups, items' groups consecutive
  const int32_t* item_order;     // [nitems] launch order of the items (largest first)
  const int32_t* item_ebox;      // [nitems] box of each work item
  const int64_t* item_gbeg;      // [nitems + 1] group range of each item
  const int64_t* item_yoff;      // [nitems] first point slot of the row partials
  const int32_t* ebox_item_beg;  // [E + 1] items of each box
  const int64_t* in_ptr;         // [E + 1] senders of column partials to each box ...
  const int64_t* in_base;        // ... and the slot of the box's first point in each
                                 //     sender's partials (senders in box order)
};

// Far-zone table on the device: launch_far_table_pgf2 for 2D-periodic kernels
// with k0 or a phase shift, launch_far_table for every other class.
struct FarTableArgs {
  int dims;         // periodic axes
  int nf[3];        // far grid nodes per axis
  double delta[3];  // far grid spacing
  double L[3];
  double k0, k0_im;
  double kt[3], kt_im[3];
  int id;           // near-zone images per periodic axis
};
void launch_far_table_pgf2(const FarTableArgs& a, void* table, hipStream_t st);
int launch_far_table(const FarTableArgs& a, bool npsp, void* table, hipStream_t st);
// The far table ([2nf-1]^3 offsets, FP64) laid out as one period of the
// circulant of length Mf >= 2 nf - 1 per axis (offset d at index d mod Mf,
// zero where no offset lands) for the FFT far sum.
void launch_far_circulant(const void* table, const int nf[3], const int Mf[3], void* out, hipStream_t st);

struct FarArgs {
  int nf[3], nint[3], nb[3];
  int64_t Ngf;
  int64_t nboxes;
};

template <typename R>
void launch_pack(const void* qu, void* qint, const int32_t* perm, int64_t N, int nrhs, int P, bool real_in,
                 bool use_perm, hipStream_t st);

// Position gradient (kernels_grad.hip): differentiated interpolation of a
// grid field F, out[m][c] += sum_p Re(conj(coef[m][p]) dF/dr_c(r_m)); and the
// correction entries differentiated on the fly (q, g packed planes).
template <typename R>
int launch_interp_grad(int q, const GridArgs& g, const double h[3], const int32_t* s3, const double* u3, int64_t N,
                       const void* grid, int P, const void* coef, double* out, hipStream_t st);
int launch_corr_grad(int q, bool cplx_vals, const CorrArgs& a, const int32_t* s3, const double* u3, const double h[3],
                     const double* pos3, const int32_t* box_start, const void* g0tab, int P, const void* qint,
                     const void* gint, bool single, double* out, hipStream_t st);
// [N][3] doubles from plan order to the caller's order (use_perm) or copied.
void launch_unpermute3(const double* in, const int32_t* perm, int64_t N, bool use_perm, double* out, hipStream_t st);
// Up to three part buffers summed elementwise in a fixed order (null = absent).
template <typename R>
struct PartPtrs {
  const cplx<R>* a;
  const cplx<R>* b;
  const cplx<R>* c;
  const cplx<R>* self;  // packed input of a diagonal term coef * input (null: none)
  R cr, ci;             // its coefficient
  __device__ cplx<R> sum(int64_t i) const {
    cplx<R> s = cmake<R>(R(0), R(0));
    if (a) s = cadd(s, a[i]);
    if (b) s = cadd(s, b[i]);
    if (c) s = cadd(s, c[i]);
    if (self) s = cadd(s, cmul(cmake<R>(cr, ci), self[i]));
    return s;
  }
};

// A diagonal term coef * x (x the packed input of the apply) added after the
// parts: the "exclude self" option subtracts lim_{r->0}[G^p - G0] q_m.
struct DiagTerm {
  const void* in = nullptr;
  double re = 0.0, im = 0.0;
};

template <typename R>
void launch_unpack(const void* u_near, const void* u_corr, const void* u_far, void* uu, const int32_t* perm,
                   int64_t N, int nrhs, int P, bool real_out, bool use_perm, const double* mean, hipStream_t st,
                   DiagTerm diag = DiagTerm());
// work: plane_sums_chunks(N) * P * 4 doubles of scratch
int64_t plane_sums_chunks(int64_t N);
template <typename R>
void launch_plane_sums(const void* a, const void* b, const void* c, int64_t N, int P, double* work, double* out,
                       hipStream_t st, DiagTerm diag = DiagTerm());
void launch_check_neutral(const double* sums, int P, double tol, int* status, hipStream_t st);
void launch_mean_from_sums(const double* sums, int P, int64_t N, double* mean, hipStream_t st);
// Projection through the node-major weight CSR (few planes).
template <typename R>
void launch_spread_csr(const int64_t* wnode, int64_t nnodes, const int64_t* wrow, const int32_t* widx,
                       const double* wval, int64_t n3, const void* qint, int P, void* grid, hipStream_t st);
template <typename R>
int launch_spread_near(int q, const GridArgs& g, const int32_t* box_start, const int32_t* s3, const double* u3,
                       int64_t N, const void* qint, int P, void* grid, hipStream_t st);
template <typename R>
int launch_interp(int q, const GridArgs& g, const int32_t* s3, const double* u3, int64_t N, const void* grid,
                  int P, void* uint, bool acc, hipStream_t st);
template <typename R>
void launch_fft_pass(int mode, const void* in, void* out, const FftPassDesc& d, const void* tw,
                     const void* spec, bool conj_spec, hipStream_t st);
void launch_near_table(void* T, const NearTableArgs& a, hipStream_t st);
template <typename R>
void launch_scale_convert(const void* in, void* out, int64_t n, double s, hipStream_t st);

// correction
int launch_corr_count(const CorrArgs& a, const int32_t* s3, const int32_t* box_start, int64_t* rowcount,
                      hipStream_t st);
// rows: s3/u3/pos3 ([3][a.N]); columns: u3c/pos3c ([3][a.Nc]) and box_start
int launch_corr_fill(int q, bool cplx_vals, bool adj, const CorrArgs& a, const int32_t* s3, const double* u3,
                     const double* pos3, const double* u3c, const double* pos3c, const int32_t* box_start,
                     const void* g0tab, const int64_t* rowptr, int32_t* col, void* val, void* val_adj,
                     hipStream_t st);
// Dense row tiles of real correction values (see kernels_corr.hip).
void launch_tile_fill(const int32_t* tile_rows, int64_t nslots, const int64_t* rowptr, const int32_t* col,
                      const double* val, const int64_t* coff, const int32_t* cols, const int64_t* voff, double* tv,
                      hipStream_t st);
template <typename R>
void launch_corr_tile(const int32_t* tile_rows, int64_t ntiles, const int64_t* coff, const int32_t* cols,
                      const int64_t* voff, const double* tv, const void* x, int P, void* u, hipStream_t st);
// order (optional, nslots entries, -1 = idle slot): the row processed by each
// wavefront slot, grouped so that a workgroup's rows are spatially close.
template <typename R>
void launch_corr_spmv(bool cplx_vals, const int64_t* rowptr, const int32_t* col, const void* val, int64_t N,
                      const int32_t* order, int64_t nslots, const void* qint, int P, void* uint, bool accumulate,
                      hipStream_t st);
int launch_sym_fill(int q, bool cplx_vals, const SymArgs& a, const double* w3, const double* pos3,
                    const void* g0tab, void* vals, hipStream_t st);
template <typename R>
void launch_sym_apply(bool cplx_vals, const SymArgs& a, const void* vals, const void* x1, const void* x2, int P1,
                      int P, bool conj1, bool conj2, void* ypart, void* zpart, void* u1, void* u2, bool accumulate,
                      hipStream_t st);

// far zone
template <typename R>
int launch_far_moments(int qf, const FarArgs& f, const int32_t* fbox_start, const int32_t* fperm,
                       const double* u3, int64_t N, const void* qint, int P, void* mom, hipStream_t st);
template <typename R>
int launch_far_gather(int qf, const FarArgs& f, const void* mom, int P, void* grid, hipStream_t st);
// the far grid sum splits its inner dimension over this many blocks
int far_apply_splits(int64_t Ngf, int P);
// Far-zone interpolation staged per far box (batched planes); returns false
// (nothing launched) when the case is not covered, e.g. few planes.
template <typename R>
bool launch_far_interp_box(int qf, const FarArgs& f, const int32_t* fbox_start, const int32_t* fperm, int max_box,
                           const int32_t* s3, const double* w3, int64_t N, const void* grid, int P, void* u, bool acc,
                           hipStream_t st);
template <typename R>
void launch_far_apply(const FarArgs& f, const void* table, const void* in, void* out, void* part, int P,
                      bool adjoint, int bf16_in, hipStream_t st);

}  // namespace fftpim
