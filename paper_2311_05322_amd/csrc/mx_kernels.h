// Host-callable launchers of the gfx950 kernels (all enqueue on stream s).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

namespace mx {

template <typename R> struct cplx_t;
template <typename R> using C_t = typename cplx_t<R>::type;

// Kernel classes (same numbering as the MX_K_* enum of mx.h).
enum KClass {
  K_LU_PANEL = 0, K_LU_ROWPANEL = 1, K_LU_UPDATE = 2, K_LU_INV = 3, K_TRSM_LOWER = 4, K_TRSM_UPPER = 5,
  K_SPMM = 6, K_RESTRICT = 7, K_PROLONG = 8, K_CGS = 9, K_ASSEMBLE = 10, K_LOCAL = 11, K_COARSE = 12,
  K_NCLASS = 16
};

// Optional launch bracketing used for per-kernel-class device timing.
struct KTimer {
  virtual void begin(int cls) = 0;
  virtual void end(int cls) = 0;
  virtual ~KTimer() {}
};

// operator assembly
void launch_element(hipStream_t s, int32_t nt, const int32_t* ts, const double* xyz, const double2* eps,
                    int eps_kind, double k0sq, double2* out);
void launch_face(hipStream_t s, int32_t n, const int32_t* ftet, const int32_t* flf, const int32_t* ts,
                 const double* xyz, const double2* eps, int eps_kind, int per_tet_k, double k0, double2 kconst,
                 double2* out, const double2* kface = nullptr);
// metallic (PEC) edge elimination in the CSR operator and the dense subdomain
// matrices, and zeroing of metallic rows of a block right-hand side
void launch_pec_csr(hipStream_t s, int64_t n, const int64_t* rp, const int32_t* col, const int32_t* pec,
                    double2* val);
template <typename C>
void launch_pec_local(hipStream_t s, int32_t nsub, const int32_t* Npad, const int64_t* mat_off, const int64_t* ptr,
                      const int32_t* idx, C* A);
void launch_zero_rows(hipStream_t s, int64_t n, const int32_t* rows, int nrhs, double2* B);
void launch_gather_csr(hipStream_t s, int64_t n, const int64_t* ptr, const int32_t* src, const double2* pool,
                       double2* out);
template <typename C>
void launch_gather_dense(hipStream_t s, int64_t n, const int64_t* dest, const int64_t* ptr, const int32_t* src,
                         const double2* pool, C* out);
template <typename C> void launch_fill_zero(hipStream_t s, int64_t n, C* out);
// the factor tiles inside the extents ext_l / ext_u ([nsub][np]) recorded by
// the last completed factorisation set back to zero
template <typename C>
void launch_clear_envelope(hipStream_t s, int32_t nsub, int np, const int32_t* Npad, const int64_t* mat_off,
                           const int32_t* ext_l, const int32_t* ext_u, C* A);
template <typename C>
void launch_pad_identity(hipStream_t s, int32_t nsub, const int64_t* dof_ptr, const int32_t* Npad,
                         const int64_t* mat_off, C* A);

// adjoint gradient
void launch_grad_tet(hipStream_t s, int32_t nt, const int32_t* ts, const double* xyz, const int32_t* t2e,
                     const double2* lam, const double2* u, int nrhs, const double2* eps, double k0sq, double2* gt,
                     double2* rt);
void launch_grad_vertex(hipStream_t s, int32_t nv, const int64_t* v2t_ptr, const int32_t* v2t, const int32_t* ts,
                        const double2* gt, const double2* rt, double reg, double2* grad, double2* keps);

// learned coarse correction
void launch_coarse_P(hipStream_t s, int64_t nrows, const int32_t* row_sub, const int32_t* dofs, const int32_t* edges,
                     const double* xyz, const double* box, float* P);
void launch_pool(hipStream_t s, int nsub, const int64_t* dof_ptr, const int32_t* dofs, const float* P,
                 const double* wts, const double2* v, int nrhs, const double* scale, float* X, float* part);
// floats of the partial-sum scratch launch_pool needs (part)
int64_t pool_scratch_floats(int nsub);
template <typename C>
void launch_coarse_apply(hipStream_t s, int64_t nrows, const int32_t* lpos, const int64_t* dof_ptr,
                         const int64_t* vec_off, const float* P, const float* Cn, int nsub, int nrhs,
                         const double* scale, float alpha, C* xloc);
void launch_gapply(hipStream_t s, int nsub, int nrhs, const double* G, const float* in, float* out);
void launch_pdp(hipStream_t s, int nsub, const int64_t* dof_ptr, const float* P, const double* D, double* out);
void launch_gemm(hipStream_t s, bool ta, bool tb, int M, int N, int K, const float* A, int lda, const float* B,
                 int ldb, float* C, int ldc, int beta, const float* bias, int act, float* Z, int rnd, int nsplit,
                 float* work);
void launch_nbr_mean(hipStream_t s, int ngraph, int nsub, int F, const int64_t* nptr, const int32_t* nbrs,
                     const float* in, float* out);
void launch_nbr_mean_T(hipStream_t s, int ngraph, int nsub, int F, const int64_t* nptr, const int32_t* nbrs,
                       const float* in, float* out, int accumulate);
void launch_gelu_back(hipStream_t s, int64_t n, const float* dh, const float* z, float* dz);
int mse_blocks();
void launch_mse(hipStream_t s, int64_t n, const float* out, const float* y, float* d, double* part);
void launch_colsum(hipStream_t s, int rows, int F, const float* in, float* out);
void launch_adam(hipStream_t s, int64_t n, float* w, const float* g, float* m, float* v, float lr, float b1, float b2,
                 float eps, int t);
void launch_gather_rows(hipStream_t s, int nrows_out, int F, const int32_t* graphs, int nsub, const float* src,
                        float* dst);
void launch_scale_f(hipStream_t s, int64_t n, float* x, float f);
void launch_nonfinite(hipStream_t s, int64_t n, const float* x, int32_t* flag);

// operator application and Schwarz transfer
// Column windows of the rows for SpMM variant 2 (slices of at most
// kSpmmWinRows consecutive rows touching at most kSpmmWinCap columns):
// srow/scp [nsl+1] first row and ucol offset of each slice, ucol the slice's
// columns, lcol [nnz] position of each non-zero's column in its slice's list.
constexpr int kSpmmWinCap = 128, kSpmmWinRows = 32;
struct SpmmWindows {
  int32_t nsl;
  const int32_t* srow;
  const int32_t* scp;
  const int32_t* ucol;
  const uint8_t* lcol;
};
// variant 0: one lane per right-hand side; 1: 32 lanes per row, entries
// broadcast (nrhs <= 32); 2: column windows staged in LDS (needs win)
void launch_spmm(hipStream_t s, int64_t nrows, const int64_t* rp, const int32_t* col, const double2* val,
                 const double2* X, double2* Y, int nrhs, int variant = 0, const SpmmWindows* win = nullptr);
template <typename C>
void launch_restrict(hipStream_t s, int64_t nrows, const int32_t* rowsrc, const double2* v, C* xloc, int nrhs);
// z[e] = sum over the entries of edge e (ptr [ne+1]) of w * zloc[row]
template <typename C>
void launch_prolong(hipStream_t s, int64_t ne, const int64_t* ptr, const int64_t* row, const double* w,
                    const C* zloc, double2* z, int nrhs,
                    double2* z2 = nullptr, int64_t ld2 = 0);

// dense subdomain factorisation and solves
// Band bookkeeping of the factorisation (device arrays, np = N_max / 64 per
// subdomain): ext_l[s*np + p] = last 64-row tile with a non-zero in the L
// part of panel p, ext_u[s*np + p] = last 64-column tile with a non-zero in
// its U part (p itself when there is none); tptr [nsub+1] / tbox [2 nsub]:
// tile lists of one trailing update; work[0]: 64x64x64 complex tile products
// of the factorisation.
// band0[s*np + p]: last row tile with a structural non-zero in the columns
// of panel p before elimination; lim[3s..3s+2]: rows [k, lim0) of the current
// panel that can hold non-zeros and the columns [lim2, lim1) its rows can.
struct LuBand {
  int32_t* ext_l;
  int32_t* ext_u;
  int64_t* tptr;
  int32_t* tbox;
  int64_t* work;
  const int32_t* band0;
  int32_t* lim;
  int np;
};
// panel_rows[p]: bound on the rows from panel p's first row that can hold
// non-zeros in its columns, over all subdomains (from the structural band);
// status[s] < 0 reports a panel whose rows exceeded it; group: panels per
// trailing-update pass (>= 1)
template <typename R>
void launch_lu(hipStream_t st, C_t<R>* pool, const int64_t* mat_off, const int32_t* Npad, const int32_t* order,
               int32_t* piv, const int64_t* vec_off, int32_t* status, int32_t* pswap,
               const std::vector<int32_t>& Nsorted, const LuBand& band, const std::vector<int32_t>& panel_rows,
               int group, KTimer* tm);
void launch_perm(hipStream_t st, int32_t nsub, const int32_t* Npad, const int64_t* vec_off, const int32_t* dense_edge,
                 const int32_t* piv, int32_t* perm_scratch, int32_t* rowsrc);
template <typename R>
// trs_lo[s*np + t]: first 64-column tile of row tile t's L part; trs_hi: last
// column tile of its U part (from the band bookkeeping of the factorisation);
// cols: right-hand-side columns per workgroup (16 or 32)
void launch_trsm(hipStream_t st, const C_t<R>* pool, const int64_t* mat_off, const int32_t* Npad,
                 const int64_t* vec_off, const int32_t* order, C_t<R>* xloc, int nsub, int nrhs,
                 const int32_t* trs_lo, const int32_t* trs_hi, int np, int cols, KTimer* tm);
int lu_max_swap_rows();

// Krylov
int dot_blocks(int64_t nrows);
void launch_dot(hipStream_t s, int64_t nrows, int nrhs, const double2* V, int64_t vstride, int nvec,
                const double2* w, double2* part, double2* out);
// w <- w - V h (nv basis vectors; skipped when h == NULL), then hout = V^H w
// (hout != NULL) or nout = ||w|| per column (hout == NULL); nv, nrhs <= 32;
// returns -1 otherwise
int cgs_fused_max();
int launch_cgs_pass(hipStream_t s, int64_t nrows, int nrhs, const double2* V, int64_t vstride, int nv,
                    const double2* h, double2* w, double2* part, double* npart, double2* hout, double* nout);
void launch_update(hipStream_t s, int64_t nrows, int nrhs, const double2* V, int64_t vstride, int nv,
                   const double2* h, double2* w);
void launch_norm(hipStream_t s, int64_t nrows, int nrhs, const double2* w, double* part, double* out);
void launch_scale(hipStream_t s, int64_t nrows, int nrhs, const double2* src, const double* nrm, double2* dst);
void launch_bminus(hipStream_t s, int64_t n, const double2* b, double2* r);
void launch_givens(hipStream_t s, int k, int m, int nrhs, const double2* h1, const double2* h2, const double* hn,
                   double2* H, double* cs, double2* sn, double2* g, const double* bnorm, double rtol, int32_t* conv,
                   int32_t* kdone, double* res);
void launch_lsq(hipStream_t s, int ksteps, int m, int nrhs, const double2* H, const double2* g, const int32_t* conv,
                int32_t* kdone, double2* y);
void launch_xupdate(hipStream_t s, int64_t nrows, int nrhs, const double2* Z, int64_t vstride, const double2* y,
                    const int32_t* kd, double2* x);
void launch_scatter_rhs(hipStream_t s, int64_t n, const int32_t* edge, const int32_t* col, const double2* val,
                        double2 scale, int nrhs, double2* B);
void launch_receivers(hipStream_t s, int nrx, int nrhs, const int64_t* ptr, const int32_t* edge, const double2* val,
                      const double2* U, double2* S);

// block FGMRES products (k_block.hip); s <= 32 columns per block
int64_t block_partial_max(int ka_max, int s);
void launch_bdot(hipStream_t st, int64_t nrows, int ka, int s, const double2* A, int64_t lda, const double2* B,
                 int64_t ldb, double2* P, double2* out);
// (Wout2, ldwout2: an optional second destination of the same result)
void launch_bupd(hipStream_t st, int64_t nrows, int ka, int s, const double2* A, int64_t lda, const double2* H,
                 const double2* Win, int64_t ldwin, double2* Wout, int64_t ldwout, double alpha, double beta,
                 double2* Wout2 = nullptr, int64_t ldwout2 = 0);
void launch_bcopy(hipStream_t st, int64_t nrows, int s, const double2* src, int64_t lds, double2* dst, int64_t ldd);

}  // namespace mx
