// Batched dense complex LU with partial pivoting of all subdomain matrices and
// the batched multi-right-hand-side triangular solves, templated on the real
// type (double: complex128 factors, float: complex64 factors on MFMA).
//
// Storage: subdomain s owns a row-major N_s x N_s block at pool + mat_off[s];
// N_s is a multiple of NB = 64 (rows/columns past the real size hold an
// identity).  The factorisation is P A = L U in LAPACK form (pivot k swaps
// rows k and piv[k] across all columns).  On exit the diagonal 64x64 blocks
// hold inverses: strictly lower part = strictly lower part of L_bb^{-1}
// (unit diagonal implied), upper part incl. diagonal = U_bb^{-1}; the other
// blocks hold L (below) and U (above).  The triangular solves then consist of
// matrix products only, which run on the 16x16x4 matrix cores.
//
// One factorisation is a sequence of launches per 64-column panel:
//   k_lu_panel     one 1024-thread workgroup per matrix: left-looking
//                  factorisation of the 64-wide panel in register-resident
//                  sub-panels of W columns, partial pivoting by workgroup
//                  reduction, then L11 -> L11^{-1} in place and the composed
//                  row permutation of the panel;
//   k_lu_rowpanel  applies the permutation to the columns outside the panel
//                  and forms U12 = L11^{-1} A12 (MFMA); k_lu_rowswap the
//                  permutation alone;
//   k_lu_update    A22 -= L21 U12 on 64x64 tiles (MFMA, LDS-staged operands),
//                  the trailing matrix once per group of panels (group
//                  size a launch parameter, picked by the autotuner).
#include "mx_device.h"
#include "mx_kernels.h"

namespace mx {

namespace {

constexpr int NB = 64;
// panels per pass over the trailing matrix (1M chamber, complex64 update:
// 2 -> 1.54 s, 4 -> 1.44 s, 8 -> 1.38 s, 16 -> 1.37 s per factorisation)
constexpr int PT = 1024;     // panel workgroup size
constexpr int MAXSW = 128;   // max distinct rows touched by one panel's swaps

// register sub-panel width of k_lu_panel by rows per thread (fewer, wider
// sub-panels: fewer top-row solves and L re-reads). 1M chamber, panels per
// factorisation: complex64 W = 4 -> 71.6 ms, 8 -> 63.4 ms, 16 -> 60.5 ms;
// complex128 W = 2 -> 121.5 ms, 4 -> 93.6 ms, 8 -> 81.7 ms. The wider widths
// fit the 128-register budget of a 1,024-thread workgroup only with one row
// per thread (32 / 16 columns spill there; 16 / 8 spill with more rows).
template <typename R, int RPT> struct PanelW;
template <int RPT> struct PanelW<float, RPT> { static constexpr int W = RPT == 1 ? 16 : 8; };
template <int RPT> struct PanelW<double, RPT> { static constexpr int W = RPT == 1 ? 8 : 4; };

template <typename R> __device__ inline Acc_t<R> zacc() {
  Acc_t<R> z;
  z[0] = 0; z[1] = 0; z[2] = 0; z[3] = 0;
  return z;
}
template <typename C> __device__ inline C czero() { C z; z.x = 0; z.y = 0; return z; }
template <typename C, typename R> __device__ inline C make_c(R re, R im) { C z; z.x = re; z.y = im; return z; }
template <typename C> __device__ inline C cone() { C z; z.x = 1; z.y = 0; return z; }
template <typename C> __device__ inline C cmulT(C a, C b) {
  C z; z.x = a.x * b.x - a.y * b.y; z.y = a.x * b.y + a.y * b.x; return z;
}
template <typename C> __device__ inline C csubT(C a, C b) { C z; z.x = a.x - b.x; z.y = a.y - b.y; return z; }
template <typename C> __device__ inline C crecip(C a) {
  C one = cone<C>();
  return cdiv(one, a);
}

// value of v in lane i (i wave-uniform)
__device__ inline float read_lane(float v, int i) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), i));
}
__device__ inline double read_lane(double v, int i) {
  const int64_t b = __double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)b, i);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(b >> 32), i);
  return __longlong_as_double((int64_t)(((uint64_t)hi << 32) | lo));
}

// --------------------------------------------------------------------------
// panel factorisation
// --------------------------------------------------------------------------
template <typename R, int RPT>
__global__ void __launch_bounds__(PT) k_lu_panel(C_t<R>* __restrict__ pool, const int64_t* __restrict__ mat_off,
                                                 const int32_t* __restrict__ Npad, const int32_t* __restrict__ order,
                                                 int32_t* __restrict__ piv, const int64_t* __restrict__ vec_off,
                                                 int32_t* __restrict__ status, int32_t* __restrict__ pswap,
                                                 const int32_t* __restrict__ lim, int k0) {
  typedef C_t<R> C;
  constexpr int W = PanelW<R, RPT>::W;
  const int s = order[blockIdx.x];
  const int N = Npad[s];
  if (k0 >= N) return;
  // rows at and beyond Nr are zero in the panel's columns (band bookkeeping):
  // they are neither read nor written, and never a pivot
  const int Nr = lim[3 * s];
  C* A = pool + mat_off[s];
  int32_t* pv = piv + vec_off[s];
  // the launch holds PT * RPT rows from k0 (chosen on the host from the
  // structural band, which bounds Nr); rows beyond would be skipped, so a
  // bound that does not hold is reported (negative status) instead
  if (threadIdx.x == 0 && Nr - k0 > PT * RPT) status[s] = -(k0 + 1);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;

  __shared__ C Utop[NB][W];
  __shared__ C swp[2][W];
  __shared__ R red_v[PT / 64];
  __shared__ int red_r[PT / 64];
  __shared__ int piv_row;
  __shared__ R piv_abs;
  __shared__ int spv[PanelW<R, RPT>::W];
  __shared__ C Lt[NB][NB + 1];
  __shared__ C Xt[NB][NB + 1];
  __shared__ int sw_dst[MAXSW], sw_src[MAXSW];
  __shared__ int sw_n;

  C a[RPT][W];
  for (int s0 = 0; s0 < NB; s0 += W) {
    const int c0 = k0 + s0;
    // (A) top rows of the sub-panel columns: U[k0:c0, c0:c0+W] = L11^{-1} A by
    // forward substitution, one wave per column, lane l holding row l. L11
    // rows are final once their pivots are taken, so the rows of the
    // previous sub-panel are copied into Lt here.
    if (s0 > 0)
      for (int e = tid; e < W * s0; e += PT) {
        const int i = s0 - W + e / s0, l = e % s0;
        if (l < i) Lt[i][l] = A[(int64_t)(k0 + i) * N + k0 + l];
      }
    __syncthreads();
    if (wv < W && s0 > 0) {
      // column-oriented: lane l holds row l of the right-hand side; at step
      // i row i is final, its value is broadcast with readlane and the rows
      // below subtract L[l][i] x_i (no reduction per step)
      const int cc = c0 + wv;
      C b = lane < s0 ? A[(int64_t)(k0 + lane) * N + cc] : czero<C>();
      for (int i = 0; i < s0; ++i) {
        const C xi = make_c<C>(read_lane(b.x, i), read_lane(b.y, i));
        if (lane > i && lane < s0) b = csubT(b, cmulT(Lt[lane][i], xi));
      }
      if (lane < s0) {
        Utop[lane][wv] = b;
        A[(int64_t)(k0 + lane) * N + cc] = b;
      }
    }
    __syncthreads();
    // (B) load sub-panel rows [c0, N) and subtract L[r, k0:c0] U[k0:c0, sub]
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = c0 + tid + PT * i;
      if (r < Nr) {
        const C* row = A + (int64_t)r * N;
#pragma unroll
        for (int j = 0; j < W; ++j) a[i][j] = row[c0 + j];
        // whole 128-byte lines of L per step (the row segment starts on a
        // line: N and k0 are multiples of 64), half lines with 8 rows per
        // thread (register budget), then W entries at a time
        constexpr int LQ = RPT <= 4 ? 128 / (int)sizeof(C) : 64 / (int)sizeof(C);
        int l = 0;
        for (; l + LQ <= s0; l += LQ) {
          C lv[LQ];
#pragma unroll
          for (int q = 0; q < LQ; ++q) lv[q] = row[k0 + l + q];
#pragma unroll
          for (int q = 0; q < LQ; ++q)
#pragma unroll
            for (int j = 0; j < W; ++j) a[i][j] = csubT(a[i][j], cmulT(lv[q], Utop[l + q][j]));
        }
        for (; l < s0; l += W) {
          C lv[W];
#pragma unroll
          for (int q = 0; q < W; ++q) lv[q] = row[k0 + l + q];
#pragma unroll
          for (int q = 0; q < W; ++q)
#pragma unroll
            for (int j = 0; j < W; ++j) a[i][j] = csubT(a[i][j], cmulT(lv[q], Utop[l + q][j]));
        }
      }
    }
    // (C) factor the W columns with partial pivoting (unrolled: a[][] is
    // indexed with constants only, so it stays in registers)
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const int c = c0 + j;
      R best = -1;
      int brow = 0x7fffffff;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = c0 + tid + PT * i;
        if (r < Nr && r >= c) {
          R v = fabs(a[i][j].x) + fabs(a[i][j].y);
          if (v > best || (v == best && r < brow)) { best = v; brow = r; }
        }
      }
      for (int off = 32; off >= 1; off >>= 1) {
        R ob = __shfl_xor(best, off);
        int orow = __shfl_xor(brow, off);
        if (ob > best || (ob == best && orow < brow)) { best = ob; brow = orow; }
      }
      if (lane == 0) { red_v[wv] = best; red_r[wv] = brow; }
      __syncthreads();
      if (tid == 0) {
        R b = red_v[0];
        int br = red_r[0];
        for (int w = 1; w < PT / 64; ++w)
          if (red_v[w] > b || (red_v[w] == b && red_r[w] < br)) { b = red_v[w]; br = red_r[w]; }
        // no usable pivot (zero or non-finite column): keep the row order so
        // every later access stays inside the matrix, and report the column
        if (!(b > 0) || br < c || br >= Nr) {
          br = c;
          b = 0;
          if (status[s] == 0) status[s] = c + 1;
        }
        piv_row = br;
        piv_abs = b;
        spv[j] = br;
      }
      __syncthreads();
      const int p = piv_row;
      // swap rows c and p: registers of the sub-panel ...
      const int oc = c - c0, op = p - c0;
      if ((oc % PT) == tid) {
#pragma unroll
        for (int i = 0; i < RPT; ++i)
          if (i == oc / PT)
#pragma unroll
            for (int jj = 0; jj < W; ++jj) swp[0][jj] = a[i][jj];
      }
      if ((op % PT) == tid) {
#pragma unroll
        for (int i = 0; i < RPT; ++i)
          if (i == op / PT)
#pragma unroll
            for (int jj = 0; jj < W; ++jj) swp[1][jj] = a[i][jj];
      }
      // ... and the other columns of the panel in memory
      if (p != c && tid < NB) {
        const int col = k0 + tid;
        if (col < c0 || col >= c0 + W) {
          C t0 = A[(int64_t)c * N + col];
          A[(int64_t)c * N + col] = A[(int64_t)p * N + col];
          A[(int64_t)p * N + col] = t0;
        }
      }
      __syncthreads();
      if ((oc % PT) == tid) {
#pragma unroll
        for (int i = 0; i < RPT; ++i)
          if (i == oc / PT)
#pragma unroll
            for (int jj = 0; jj < W; ++jj) a[i][jj] = swp[1][jj];
      }
      if ((op % PT) == tid && p != c) {
#pragma unroll
        for (int i = 0; i < RPT; ++i)
          if (i == op / PT)
#pragma unroll
            for (int jj = 0; jj < W; ++jj) a[i][jj] = swp[0][jj];
      }
      // eliminate below the pivot (pivot row values are swp[1])
      const bool ok = piv_abs > 0;
      C inv = ok ? crecip(swp[1][j]) : czero<C>();
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = c0 + tid + PT * i;
        if (r < Nr && r > c) {
          C l = cmulT(a[i][j], inv);
          a[i][j] = l;
#pragma unroll
          for (int jj = j + 1; jj < W; ++jj) a[i][jj] = csubT(a[i][jj], cmulT(l, swp[1][jj]));
        }
      }
      __syncthreads();
    }
    // (D) write the sub-panel back
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = c0 + tid + PT * i;
      if (r < Nr) {
#pragma unroll
        for (int j = 0; j < W; ++j) A[(int64_t)r * N + c0 + j] = a[i][j];
      }
    }
    if (tid < W) pv[c0 + tid] = spv[tid];
    __syncthreads();
  }
  // ---- L11 -> L11^{-1} (unit lower, strictly lower part stored)
  for (int e = tid; e < NB * NB; e += PT) {
    int i = e / NB, j = e % NB;
    Lt[i][j] = A[(int64_t)(k0 + i) * N + k0 + j];
  }
  __syncthreads();
  if (tid < NB) {
    // column j of X = L^{-1}: X[j][j] = 1, X[i][j] = -sum_{l=j}^{i-1} L[i][l] X[l][j]
    const int j = tid;
    Xt[j][j] = cone<C>();
    for (int i = j + 1; i < NB; ++i) {
      C acc = czero<C>();
      for (int l = j; l < i; ++l) acc = csubT(acc, cmulT(Lt[i][l], Xt[l][j]));
      Xt[i][j] = acc;
    }
  }
  __syncthreads();
  for (int e = tid; e < NB * NB; e += PT) {
    int i = e / NB, j = e % NB;
    if (j < i) A[(int64_t)(k0 + i) * N + k0 + j] = Xt[i][j];
  }
  // ---- composed permutation of this panel's swaps (rows >= k0)
  if (tid == 0) {
    int n = NB;
    for (int k = 0; k < NB; ++k) { sw_dst[k] = k0 + k; sw_src[k] = k0 + k; }
    for (int k = 0; k < NB; ++k) {
      const int p = pv[k0 + k];
      if (p == k0 + k) continue;
      int ib = -1;
      if (p < k0 + NB) {
        ib = p - k0;
      } else {
        for (int q = NB; q < n; ++q)
          if (sw_dst[q] == p) { ib = q; break; }
        if (ib < 0) { ib = n++; sw_dst[ib] = p; sw_src[ib] = p; }
      }
      int t = sw_src[k];
      sw_src[k] = sw_src[ib];
      sw_src[ib] = t;
    }
    sw_n = n;
  }
  __syncthreads();
  int32_t* ps = pswap + (int64_t)s * (2 * MAXSW + 1);
  if (tid == 0) ps[0] = sw_n;
  for (int q = tid; q < sw_n; q += PT) {
    ps[1 + q] = sw_dst[q];
    ps[1 + MAXSW + q] = sw_src[q];
  }
}

// --------------------------------------------------------------------------
// row permutation outside the panel and U12 = L11^{-1} A12.
// mode 0: both; mode 1: the permutation only (all rows written back);
// mode 2: U12 only, from the rows k0..k0+63 as they stand (the permutation
// already applied and any deferred update of those rows already done).
// --------------------------------------------------------------------------
template <typename R, int XR>
__global__ void __launch_bounds__(256) k_lu_rowpanel(C_t<R>* __restrict__ pool, const int64_t* __restrict__ mat_off,
                                                     const int32_t* __restrict__ Npad,
                                                     const int32_t* __restrict__ order,
                                                     const int32_t* __restrict__ pswap,
                                                     const int32_t* __restrict__ lim, int k0, int mode) {
  typedef C_t<R> C;
  typedef Acc_t<R> Acc;
  const int s = order[blockIdx.y];
  const int N = Npad[s];
  const int cb = blockIdx.x * NB;
  if (cb >= N || cb == k0 || k0 >= N) return;
  if (mode == 2 && cb < k0) return;
  // outside [lim2, lim1) every row the panel touches is zero: nothing moves
  // and U12 is zero there
  if (cb >= lim[3 * s + 1] || cb < lim[3 * s + 2]) return;
  C* A = pool + mat_off[s];
  const int32_t* ps = pswap + (int64_t)s * (2 * MAXSW + 1);
  const int n = mode == 2 ? NB : ps[0];
  // XR rows of staging: MAXSW for the permutation modes, NB for mode 2 (half
  // the LDS, so twice the workgroups per CU)
  __shared__ C X[XR][NB + 1];
  const int tid = threadIdx.x;
  // staging: eight loads per thread in flight before their LDS writes
  // (complex64; complex128 keeps one at a time, its register allocation
  // otherwise spills)
  constexpr int SU = sizeof(R) == 4 ? 8 : 1;
  for (int e0 = 0; e0 < n * NB; e0 += 256 * SU) {
    C t[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int e = e0 + tid + 256 * u;
      if (e < n * NB) {
        const int q = e / NB, j = e % NB;
        const int src = mode == 2 ? k0 + q : ps[1 + MAXSW + q];
        t[u] = A[(int64_t)src * N + cb + j];
      }
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int e = e0 + tid + 256 * u;
      if (e < n * NB) X[e / NB][e % NB] = t[u];
    }
  }
  __syncthreads();
  if (cb < k0 || mode == 1) {
    for (int e = tid; e < n * NB; e += 256) {
      int q = e / NB, j = e % NB;
      A[(int64_t)ps[1 + q] * N + cb + j] = X[q][j];
    }
    return;
  }
  // rows below the panel that received another row's content
  for (int e = tid; mode == 0 && e < (n - NB) * NB; e += 256) {
    int q = NB + e / NB, j = e % NB;
    A[(int64_t)ps[1 + q] * N + cb + j] = X[q][j];
  }
  // U12 = L11^{-1} X[0:64]; wave w computes rows 16w..16w+15, all 64 columns
  const int lane = tid & 63, w = tid >> 6;
  Acc cre[4], cim[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) { cre[ct] = zacc<R>(); cim[ct] = zacc<R>(); }
  const int ar = 16 * w + (lane & 15);
  // this lane's elements of L11^{-1} (unit lower), loaded KB steps at a time
  // before their products (all 16 for complex64, one for complex128)
  constexpr int KB = sizeof(R) == 4 ? NB / 4 : 1;
  for (int kq0 = 0; kq0 < NB / 4; kq0 += KB) {
    C avs[KB];
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      const int kcol = 4 * (kq0 + u) + (lane >> 4);
      const C v = A[(int64_t)(k0 + ar) * N + k0 + kcol];
      avs[u] = kcol < ar ? v : (kcol == ar ? cone<C>() : czero<C>());
    }
#pragma unroll
    for (int u = 0; u < KB; ++u) {
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        C bv = X[4 * (kq0 + u) + (lane >> 4)][16 * ct + (lane & 15)];
        cmfma<R>(avs[u], bv, cre[ct], cim[ct]);
      }
    }
  }
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * w + acc_row<R>(lane, r);
      C v;
      v.x = cre[ct][r];
      v.y = cim[ct][r];
      A[(int64_t)(k0 + row) * N + cb + 16 * ct + (lane & 15)] = v;
    }
}

// The permutation alone (a group's later panels): the rows ps[1+MAXSW+q]
// move to ps[1+q] in one 64-column tile outside the panel; every thread holds
// the values it moves in registers, and all reads finish (workgroup barrier)
// before any write.
template <typename R>
__global__ void __launch_bounds__(256) k_lu_rowswap(C_t<R>* __restrict__ pool, const int64_t* __restrict__ mat_off,
                                                    const int32_t* __restrict__ Npad,
                                                    const int32_t* __restrict__ order,
                                                    const int32_t* __restrict__ pswap,
                                                    const int32_t* __restrict__ lim, int k0) {
  typedef C_t<R> C;
  constexpr int PER = MAXSW * NB / 256;
  const int s = order[blockIdx.y];
  const int N = Npad[s];
  const int cb = blockIdx.x * NB;
  if (cb >= N || cb == k0 || k0 >= N) return;  // the whole workgroup
  if (cb >= lim[3 * s + 1] || cb < lim[3 * s + 2]) return;
  C* A = pool + mat_off[s];
  const int32_t* ps = pswap + (int64_t)s * (2 * MAXSW + 1);
  const int n = ps[0];
  if (n == 0) return;  // the whole workgroup
  const int tid = threadIdx.x;
  // every load unconditional (entries past the swap list repeat its first
  // row; they are not stored), so that they are all in flight together
  C v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + 256 * u;
    const int ec = e < n * NB ? e : e % NB;
    v[u] = A[(int64_t)ps[1 + MAXSW + ec / NB] * N + cb + ec % NB];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + 256 * u;
    if (e < n * NB) A[(int64_t)ps[1 + e / NB] * N + cb + e % NB] = v[u];
  }
}

// --------------------------------------------------------------------------
// trailing update A[r0.., c0..] -= A[r0.., kl..kl+kd) A[kl..kl+kd), c0..] on
// 64x64 tiles (kd = 512 for the update of the trailing matrix after a group
// of eight panels, one 512-deep pass instead of eight 64-deep ones; smaller
// kd for the in-group updates of one 64-wide column or row block), complex
// products in the 3-multiplication form (three real MFMA products instead of
// four); the panels are staged in 32-deep chunks (33.5 KB of LDS for
// complex64, 67 KB for complex128), for complex64 with the next chunk already
// in registers while the current one is multiplied; the C tile is loaded
// before the staging.
// --------------------------------------------------------------------------
constexpr int KCH = 32;

// One 64x64 tile of A22 -= L21 U12: rows i0.., columns j0.. of the matrix A
// (order N), the kd-deep product over columns kl.. of L21 and rows kl.. of
// U12. As / Bs: the workgroup's LDS staging.
template <typename R>
__device__ __forceinline__ void lu_update_tile(C_t<R>* __restrict__ A, int N, int i0, int j0, int kl, int kd,
                                               C_t<R> (&As)[NB][KCH + 1], C_t<R> (&Bs)[KCH][NB + 1]) {
  typedef C_t<R> C;
  typedef Acc_t<R> Acc;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  // C tile in registers; products accumulated in the 3-multiplication form
  // t1 = sum l.re u.re, t2 = sum l.im u.im, t3 = sum (l.re + l.im)(u.re + u.im)
  C cv[2][2][4];
#pragma unroll
  for (int it = 0; it < 2; ++it)
#pragma unroll
    for (int jt = 0; jt < 2; ++jt)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        cv[it][jt][r] = A[(int64_t)(i0 + wr + 16 * it + acc_row<R>(lane, r)) * N + j0 + wc + 16 * jt + (lane & 15)];
  Acc t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int it = 0; it < 2; ++it)
#pragma unroll
    for (int jt = 0; jt < 2; ++jt) { t1[it][jt] = zacc<R>(); t2[it][jt] = zacc<R>(); t3[it][jt] = zacc<R>(); }
  // one 4-deep step of the 3-multiplication product out of LDS
  auto mma = [&](int kk) {
    C av[2], bv[2];
    R as[2], bs[2];
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      av[it] = As[wr + 16 * it + (lane & 15)][kk + (lane >> 4)];
      as[it] = av[it].x + av[it].y;
    }
#pragma unroll
    for (int jt = 0; jt < 2; ++jt) {
      bv[jt] = Bs[kk + (lane >> 4)][wc + 16 * jt + (lane & 15)];
      bs[jt] = bv[jt].x + bv[jt].y;
    }
#pragma unroll
    for (int it = 0; it < 2; ++it)
#pragma unroll
      for (int jt = 0; jt < 2; ++jt) {
        t1[it][jt] = mfma(av[it].x, bv[jt].x, t1[it][jt]);
        t2[it][jt] = mfma(av[it].y, bv[jt].y, t2[it][jt]);
        t3[it][jt] = mfma(as[it], bs[jt], t3[it][jt]);
      }
  };
  if constexpr (sizeof(R) == 4) {
    // complex64: the next chunk's operands are loaded into registers while
    // the current chunk is multiplied out of LDS
    C ra[NB * KCH / 256], rb[NB * KCH / 256];
    auto gload = [&](int kc) {
#pragma unroll
      for (int q = 0; q < NB * KCH / 256; ++q) {
        const int e = tid + 256 * q;
        ra[q] = A[(int64_t)(i0 + e / KCH) * N + kl + kc + e % KCH];
        rb[q] = A[(int64_t)(kl + kc + e / NB) * N + j0 + e % NB];
      }
    };
    gload(0);
    for (int kc = 0; kc < kd; kc += KCH) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < NB * KCH / 256; ++q) {
        const int e = tid + 256 * q;
        As[e / KCH][e % KCH] = ra[q];
        Bs[e / NB][e % NB] = rb[q];
      }
      __syncthreads();
      if (kc + KCH < kd) gload(kc + KCH);
#pragma unroll
      for (int kk = 0; kk < KCH; kk += 4) mma(kk);
    }
  } else {
    // complex128: staged directly (the register budget holds no second chunk)
    for (int kc = 0; kc < kd; kc += KCH) {
      __syncthreads();
      for (int e = tid; e < NB * KCH; e += 256) {
        As[e / KCH][e % KCH] = A[(int64_t)(i0 + e / KCH) * N + kl + kc + e % KCH];
        Bs[e / NB][e % NB] = A[(int64_t)(kl + kc + e / NB) * N + j0 + e % NB];
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < KCH; kk += 4) mma(kk);
    }
  }
#pragma unroll
  for (int it = 0; it < 2; ++it)
#pragma unroll
    for (int jt = 0; jt < 2; ++jt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        C v = cv[it][jt][r];
        v.x -= t1[it][jt][r] - t2[it][jt][r];
        v.y -= t3[it][jt][r] - t1[it][jt][r] - t2[it][jt][r];
        A[(int64_t)(i0 + wr + 16 * it + acc_row<R>(lane, r)) * N + j0 + wc + 16 * jt + (lane & 15)] = v;
      }
}

// --------------------------------------------------------------------------
// Band bookkeeping. A subdomain matrix in reverse Cuthill-McKee order is
// banded, and elimination keeps its non-zeros near the diagonal; only 64x64
// tiles that the trailing updates can change are visited. After a panel is
// factored its L part is scanned for the last row tile holding a non-zero
// (ext_l), after its U part is formed that for the last column tile (ext_u);
// a trailing update then visits row tiles up to the largest ext_l and column
// tiles up to the largest ext_u of the panels it applies (everything beyond
// is a product with an exact zero). The row interchanges of a panel move
// values of earlier L columns between its pivot rows: an earlier panel whose
// L part reaches the current panel's rows gets its extent raised to the
// lowest pivot row. The extents are exact data (not a structural estimate),
// so they hold under any pivoting.
// --------------------------------------------------------------------------
__global__ void k_band_init(int nsub, const int32_t* __restrict__ Npad, int np, int32_t* __restrict__ ext_l,
                            int32_t* __restrict__ ext_u, int64_t* __restrict__ work) {
  const int s = blockIdx.x;
  if (s == 0 && threadIdx.x == 0) work[0] = 0;
  const int nt = Npad[s] / NB;
  for (int p = threadIdx.x; p < np; p += blockDim.x) {
    ext_l[(int64_t)s * np + p] = p < nt ? p : -1;
    ext_u[(int64_t)s * np + p] = p < nt ? p : -1;
  }
}

// wave-wide "any non-zero" over a 64-wide row segment (one value per lane)
template <typename C>
__device__ inline bool wave_any_nonzero(C v) {
  return __ballot(v.x != 0 || v.y != 0) != 0;
}

// ext_l of the panel at column k (scan of rows k+64 .. N-1, bottom up, one
// row per wave and step) and the pivot rule for the earlier panels
template <typename R>
__global__ void __launch_bounds__(256) k_band_l(const C_t<R>* __restrict__ pool, const int64_t* __restrict__ mat_off,
                                                const int32_t* __restrict__ Npad, const int32_t* __restrict__ order,
                                                const int32_t* __restrict__ piv, const int64_t* __restrict__ vec_off,
                                                int np, int32_t* __restrict__ ext_l, const int32_t* __restrict__ lim,
                                                int k) {
  const int s = order[blockIdx.x];
  const int N = Npad[s];
  if (k >= N) return;
  const C_t<R>* A = pool + mat_off[s];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __shared__ int last[4];
  int found = -1;
  for (int r = min(N, lim[3 * s]) - 1 - w; r >= k + NB; r -= 4) {
    if (wave_any_nonzero(A[(int64_t)r * N + k + lane])) {
      found = r;
      break;
    }
  }
  if (lane == 0) last[w] = found;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int p = k / NB;
    int rmax = max(max(last[0], last[1]), max(last[2], last[3]));
    int32_t* e = ext_l + (int64_t)s * np;
    e[p] = rmax >= 0 ? max(p, rmax / NB) : p;
    int pmax = k;
    for (int c = 0; c < NB; ++c) pmax = max(pmax, piv[vec_off[s] + k + c]);
    const int tm = pmax / NB;
    for (int q = 0; q < p; ++q)
      if (e[q] >= p && e[q] < tm) e[q] = tm;
  }
}

// ext_u of the panel at row k (scan of column tiles right of the panel,
// right to left, one tile per wave and step)
template <typename R>
__global__ void __launch_bounds__(256) k_band_u(const C_t<R>* __restrict__ pool, const int64_t* __restrict__ mat_off,
                                                const int32_t* __restrict__ Npad, const int32_t* __restrict__ order,
                                                int np, int32_t* __restrict__ ext_u, const int32_t* __restrict__ lim,
                                                int k) {
  const int s = order[blockIdx.x];
  const int N = Npad[s];
  if (k >= N) return;
  const C_t<R>* A = pool + mat_off[s];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __shared__ int last[4];
  const int p = k / NB;
  int found = -1;
  for (int ct = min(N, lim[3 * s + 1]) / NB - 1 - w; ct > p && found < 0; ct -= 4) {
    for (int r = 0; r < NB; ++r)
      if (wave_any_nonzero(A[(int64_t)(k + r) * N + NB * ct + lane])) {
        found = ct;
        break;
      }
  }
  if (lane == 0) last[w] = found;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int cmax = max(max(last[0], last[1]), max(last[2], last[3]));
    ext_u[(int64_t)s * np + p] = cmax >= 0 ? cmax : p;
  }
}

// Bounds of the panel at column k for every active subdomain (before it is
// factored): rows of its columns that can hold non-zeros, [k, lim0), and
// columns its rows can, [lim2, lim1). Non-zeros below the structural band
// band0 come only from earlier panels q whose L part reaches the panel's
// rows (ext_l[q] >= p): their updates (rows <= ext_l[q], columns <= ext_u[q])
// and their row interchanges (rows <= ext_l[q]); left of the panel a row
// holds L values of exactly those panels.
__global__ void __launch_bounds__(256) k_band_limits(int nact, const int32_t* __restrict__ Npad,
                                                     const int32_t* __restrict__ order, int np,
                                                     const int32_t* __restrict__ band0,
                                                     const int32_t* __restrict__ ext_l,
                                                     const int32_t* __restrict__ ext_u, int32_t* __restrict__ lim,
                                                     int k) {
  for (int z = blockIdx.x * blockDim.x + threadIdx.x; z < nact; z += gridDim.x * blockDim.x) {
    const int s = order[z];
    const int N = Npad[s];
    if (k >= N) continue;
    const int p = k / NB, nt = N / NB;
    const int32_t* el = ext_l + (int64_t)s * np;
    const int32_t* eu = ext_u + (int64_t)s * np;
    const int32_t* b0 = band0 + (int64_t)s * np;
    int re = b0[p], ce = -1, lo = p;
    for (int q = 0; q < p; ++q)
      if (el[q] >= p) {
        re = max(re, el[q]);
        ce = max(ce, eu[q]);
        lo = min(lo, q);
      }
    re = min(re, nt - 1);
    for (int t = p; t <= re; ++t) ce = max(ce, b0[t]);
    ce = min(max(ce, p), nt - 1);
    lim[3 * s] = NB * (re + 1);
    lim[3 * s + 1] = NB * (ce + 1);
    lim[3 * s + 2] = NB * lo;
  }
}

// Tile list of one trailing update A22 -= L U over the panels [pa, pb):
// mode 0 (the group's update) rows rt0 .. max ext_l, columns ct0 .. max ext_u;
// mode 1 (one panel's column block) rows rt0 .. max ext_l, column ct0 (if any
// U part reaches it); mode 2 (one panel's row block) row rt0 (if any L part
// reaches it), columns ct0 .. max ext_u. tptr = exclusive prefix of the tile
// counts over the active subdomains, tbox[2z] = first row tile,
// tbox[2z+1] = number of column tiles; work[0] += tiles * (kd / 64).
__global__ void __launch_bounds__(256) k_band_tiles(int nact, const int32_t* __restrict__ Npad,
                                                    const int32_t* __restrict__ order, int np,
                                                    const int32_t* __restrict__ ext_l,
                                                    const int32_t* __restrict__ ext_u, int pa, int pb, int rt0,
                                                    int ct0, int mode, int64_t* __restrict__ tptr,
                                                    int32_t* __restrict__ tbox, int64_t* __restrict__ work,
                                                    int kdt) {
  __shared__ int64_t part[256];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int z0 = 0; z0 < nact; z0 += 256) {
    const int z = z0 + threadIdx.x;
    int64_t cnt = 0;
    if (z < nact) {
      const int s = order[z];
      const int nt = Npad[s] / NB;
      int lmax = -1, umax = -1;
      for (int q = pa; q < pb && q < nt; ++q) {
        lmax = max(lmax, ext_l[(int64_t)s * np + q]);
        umax = max(umax, ext_u[(int64_t)s * np + q]);
      }
      lmax = min(lmax, nt - 1);
      umax = min(umax, nt - 1);
      int r1, c1;
      if (mode == 0) { r1 = lmax; c1 = umax; }
      else if (mode == 1) { r1 = lmax; c1 = umax >= ct0 ? ct0 : ct0 - 1; }
      else { r1 = lmax >= rt0 ? rt0 : rt0 - 1; c1 = umax; }
      const int nr = rt0 < nt ? max(0, r1 - rt0 + 1) : 0;
      const int nc = ct0 < nt ? max(0, c1 - ct0 + 1) : 0;
      cnt = (int64_t)nr * nc;
      tbox[2 * z] = rt0;
      tbox[2 * z + 1] = nc;
    }
    part[threadIdx.x] = cnt;
    __syncthreads();
    // inclusive scan of the block (Hillis-Steele)
    for (int o = 1; o < 256; o <<= 1) {
      const int64_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
      __syncthreads();
      part[threadIdx.x] += v;
      __syncthreads();
    }
    if (z < nact) tptr[z] = carry + part[threadIdx.x] - cnt;
    __syncthreads();
    if (threadIdx.x == 255) carry += part[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    tptr[nact] = carry;
    work[0] += carry * kdt;
  }
}

// The trailing update over a tile list: a fixed grid of workgroups walks the
// list (tile t, t + gridDim.x, ...), whatever the number of tiles; uneven
// subdomains are balanced over the whole chip.
template <typename R>
__global__ void __launch_bounds__(256, 2) k_lu_update_list(C_t<R>* __restrict__ pool, const int64_t* __restrict__ mat_off,
                                                        const int32_t* __restrict__ Npad,
                                                        const int32_t* __restrict__ order, int nact,
                                                        const int64_t* __restrict__ tptr,
                                                        const int32_t* __restrict__ tbox, int ct0, int kl, int kd) {
  typedef C_t<R> C;
  __shared__ C As[NB][KCH + 1];
  __shared__ C Bs[KCH][NB + 1];
  const int64_t total = tptr[nact];
  for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
    // subdomain of tile t: last z with tptr[z] <= t
    int lo = 0, hi = nact - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tptr[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const int z = lo;
    const int64_t loc = t - tptr[z];
    const int nc = tbox[2 * z + 1];
    const int i0 = NB * (tbox[2 * z] + (int)(loc / nc));
    const int j0 = NB * (ct0 + (int)(loc % nc));
    const int s = order[z];
    lu_update_tile<R>(pool + mat_off[s], Npad[s], i0, j0, kl, kd, As, Bs);
  }
}

// --------------------------------------------------------------------------
// U_bb -> U_bb^{-1} in the upper part of every diagonal block. Column j of
// Y = U^{-1}: Y[j][j] = 1/U[j][j], Y[i][j] = -(sum_{l=i+1}^{j} U[i][l] Y[l][j])
// / U[i][i] for i < j. Four threads per column (thread 4j + q takes the terms
// l = q mod 4, summed over the four with shuffles); one LDS array holds U in
// its upper triangle and Y transposed in its strict lower triangle (Y's
// diagonal apart), so a workgroup needs 34 KB and four fit on a compute unit.
// --------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256) k_inv_upper(C_t<R>* __restrict__ pool, const int64_t* __restrict__ mat_off,
                                                   const int32_t* __restrict__ Npad,
                                                   const int32_t* __restrict__ order) {
  typedef C_t<R> C;
  const int s = order[blockIdx.y];
  const int N = Npad[s];
  const int b0 = blockIdx.x * NB;
  if (b0 >= N) return;
  C* A = pool + mat_off[s];
  __shared__ C M[NB][NB + 1];   // M[i][l] = U[i][l] (l >= i); M[j][i] = Y[i][j] (i < j)
  __shared__ C dinv[NB];        // 1 / U[i][i] = Y[i][i]
  const int tid = threadIdx.x;
  for (int e = tid; e < NB * NB; e += 256) {
    const int i = e / NB, l = e % NB;
    if (l >= i) M[i][l] = A[(int64_t)(b0 + i) * N + b0 + l];
  }
  __syncthreads();
  if (tid < NB) dinv[tid] = crecip(M[tid][tid]);
  __syncthreads();
  const int j = tid >> 2, q = tid & 3;
  // Y[l][j] for l > i: Y[j][j] = dinv[j], otherwise M[j][l] (written below)
  for (int i = j - 1; i >= 0; --i) {
    C acc = czero<C>();
    for (int l = i + 1 + ((q - (i + 1)) & 3); l <= j; l += 4) {
      const C y = l == j ? dinv[j] : M[j][l];
      acc = csubT(acc, cmulT(M[i][l], y));
    }
    acc.x += __shfl_xor(acc.x, 1);
    acc.y += __shfl_xor(acc.y, 1);
    acc.x += __shfl_xor(acc.x, 2);
    acc.y += __shfl_xor(acc.y, 2);
    // one wave holds the four threads of column j: its LDS accesses are
    // performed in order, so the next step's read of M[j][i] sees this write
    if (q == 0) M[j][i] = cmulT(acc, dinv[i]);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  for (int e = tid; e < NB * NB; e += 256) {
    const int i = e / NB, jj = e % NB;
    if (jj > i) A[(int64_t)(b0 + i) * N + b0 + jj] = M[jj][i];
    else if (jj == i) A[(int64_t)(b0 + i) * N + b0 + i] = dinv[i];
  }
}

// rowsrc[vec_off[s] + r] = dofs[dof_ptr[s] + perm[r]] (or -1 on padded rows),
// perm = the row permutation P of P A = L U
__global__ void __launch_bounds__(64) k_perm(int32_t nsub, const int32_t* __restrict__ Npad,
                                             const int64_t* __restrict__ vec_off,
                                             const int32_t* __restrict__ dense_edge,
                                             const int32_t* __restrict__ piv, int32_t* __restrict__ perm_scratch,
                                             int32_t* __restrict__ rowsrc) {
  const int s = blockIdx.x;
  if (s >= nsub) return;
  const int N = Npad[s];
  int32_t* perm = perm_scratch + vec_off[s];
  const int32_t* pv = piv + vec_off[s];
  for (int r = threadIdx.x; r < N; r += 64) perm[r] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < N; ++k) {
      int p = pv[k];
      if (p != k) { int t = perm[k]; perm[k] = perm[p]; perm[p] = t; }
    }
  }
  __syncthreads();
  for (int r = threadIdx.x; r < N; r += 64) rowsrc[vec_off[s] + r] = dense_edge[vec_off[s] + perm[r]];
}

// --------------------------------------------------------------------------
// triangular solves: X <- U^{-1} L^{-1} X on [N][nrhs] blocks, 32 right-hand
// sides per workgroup, 256-row super-blocks, 64-row diagonal blocks applied
// through their stored inverses.
//
// Off-diagonal part of a super-block: each wave owns 16*RT rows (RT = 4 for
// complex64: four waves; RT = 2 for complex128: eight waves) and accumulates
// A[rows, K] X[K] on its own, with no workgroup barrier: it streams its
// factor rows and the matching right-hand-side rows straight into MFMA
// operand registers (complex64: the next 16-column chunk in flight while a
// chunk is multiplied); the right-hand-side rows are shared by the waves and come from
// L1/L2. Two workgroups share a compute unit for complex64; for complex128
// the workgroup's LDS admits one per compute unit, and its eight waves keep
// two on each SIMD so that one wave's loads are covered by the other's
// products. The diagonal part then runs on the super-block's residual held in
// LDS: each 64-row diagonal block is multiplied by its stored inverse and the
// remaining rows of the super-block are updated, spread over all waves in
// 16-row tiles.
// --------------------------------------------------------------------------
constexpr int SB = 256;
constexpr int KC = 16;
template <typename R> struct TrsmShape;
template <> struct TrsmShape<float> { static constexpr int RT = 4; };
template <> struct TrsmShape<double> { static constexpr int RT = 2; };
template <typename R> constexpr int trsm_waves() { return SB / (16 * TrsmShape<R>::RT); }

template <typename R, bool LOWER>
__device__ inline C_t<R> diag_inv_elem(const C_t<R>* A, int N, int b0, int i, int k) {
  typedef C_t<R> C;
  if (LOWER) {
    if (k < i) return A[(int64_t)(b0 + i) * N + b0 + k];
    return k == i ? cone<C>() : czero<C>();
  } else {
    if (k >= i) return A[(int64_t)(b0 + i) * N + b0 + k];
    return czero<C>();
  }
}

// One K chunk of operands for this lane. MFMA step s4 uses
// k = kc + 4*(lane/16) + s4: the factor row 16*rt + lane%16 is read as 4
// consecutive complex values per lane, and the right-hand-side rows with the
// same permuted k, columns 16*ct + lane%16.
template <typename R, int NCT>
struct trsm_ops {
  C_t<R> a[TrsmShape<R>::RT][4];
  C_t<R> b[4][NCT];
};

template <typename R, int NCT>
__device__ __forceinline__ void trsm_load(trsm_ops<R, NCT>& o, const C_t<R>* __restrict__ Arow, int N,
                                          const C_t<R>* __restrict__ X, int nrhs, int j0, int nc, int kc, int lane) {
#pragma unroll
  for (int rt = 0; rt < TrsmShape<R>::RT; ++rt) {
    const C_t<R>* ap = Arow + (int64_t)(16 * rt + (lane & 15)) * N + kc + 4 * (lane >> 4);
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) o.a[rt][s4] = ap[s4];
  }
  // columns beyond nc read a copy of the last column: the products of an
  // MFMA column depend on that column alone, and those columns are never
  // stored, so no branch (and no conservative wait) is needed here
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      const int col = min(16 * ct + (lane & 15), nc - 1);
      o.b[s4][ct] = X[(int64_t)(kc + 4 * (lane >> 4) + s4) * nrhs + j0 + col];
    }
}

template <typename R, int NCT>
__device__ __forceinline__ void trsm_mul3(const trsm_ops<R, NCT>& o, Acc_t<R> (&t1)[TrsmShape<R>::RT][NCT],
                                          Acc_t<R> (&t2)[TrsmShape<R>::RT][NCT],
                                          Acc_t<R> (&t3)[TrsmShape<R>::RT][NCT]) {
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4) {
    R bs[NCT];
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) bs[ct] = o.b[s4][ct].x + o.b[s4][ct].y;
#pragma unroll
    for (int rt = 0; rt < TrsmShape<R>::RT; ++rt) {
      const R as = o.a[rt][s4].x + o.a[rt][s4].y;
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) {
        t1[rt][ct] = mfma(o.a[rt][s4].x, o.b[s4][ct].x, t1[rt][ct]);
        t2[rt][ct] = mfma(o.a[rt][s4].y, o.b[s4][ct].y, t2[rt][ct]);
        t3[rt][ct] = mfma(as, bs[ct], t3[rt][ct]);
      }
    }
  }
}

// NCT: 16-column tiles of right-hand sides per workgroup (RC = 16 NCT columns);
// one workgroup per (subdomain, RC columns)
template <typename R, bool LOWER, int NCT>
__global__ void __launch_bounds__(64 * trsm_waves<R>(), (NCT == 1 && sizeof(R) == 4) ? 3 : 2)
    k_trsm(const C_t<R>* __restrict__ pool, const int64_t* __restrict__ mat_off, const int32_t* __restrict__ Npad,
           const int64_t* __restrict__ vec_off, const int32_t* __restrict__ order, C_t<R>* __restrict__ xloc,
           int nrhs, const int32_t* __restrict__ trs_lo, const int32_t* __restrict__ trs_hi, int np) {
  typedef C_t<R> C;
  typedef Acc_t<R> Acc;
  constexpr int TRT = TrsmShape<R>::RT, TNW = trsm_waves<R>();
  constexpr int RC = 16 * NCT;
  const int s = order[blockIdx.x];
  const int N = Npad[s];
  const C* A = pool + mat_off[s];
  C* X = xloc + vec_off[s] * (int64_t)nrhs;
  const int j0 = blockIdx.y * RC;
  const int nc = min(RC, nrhs - j0);
  __shared__ C Tb[SB][RC + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nsb = (N + SB - 1) / SB;
  for (int q = 0; q < nsb; ++q) {
    const int sbi = LOWER ? q : nsb - 1 - q;
    const int b0 = sbi * SB;
    const int nd = min(SB, N - b0) / NB;
    if (w < nd * (NB / (16 * TRT))) {  // this wave's rows lie in the super-block
      const C* Arow = A + (int64_t)(b0 + 16 * TRT * w) * N;
      Acc cre[TRT][NCT], cim[TRT][NCT];
#pragma unroll
      for (int rt = 0; rt < TRT; ++rt)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) { cre[rt][ct] = zacc<R>(); cim[rt][ct] = zacc<R>(); }
      // off-diagonal part over K = [kbeg, kbeg + KC * nch): the band of this
      // wave's row tile (L: from its first non-zero column tile up to the
      // super-block; U: from the super-block's end up to its last one)
      const int tw = (b0 + 16 * TRT * w) / NB;
      const int kbeg = LOWER ? NB * trs_lo[(int64_t)s * np + tw] : b0 + nd * NB;
      const int kend = LOWER ? b0 : min(N, NB * (trs_hi[(int64_t)s * np + tw] + 1));
      const int nch = max(0, (kend - kbeg) / KC);
      // chunk c of the band: L from the super-block backwards (every wave of
      // the forward solve then starts at the same right-hand-side rows, as
      // the backward solve's waves do; complex128 forward solve 6.57 ->
      // 6.30 ms, complex64 unchanged), U forwards
      auto kc_of = [&](int c) { return LOWER ? kend - (c + 1) * KC : kbeg + c * KC; };
      if (nch > 0) {
        Acc t3[TRT][NCT];
#pragma unroll
        for (int rt = 0; rt < TRT; ++rt)
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) t3[rt][ct] = zacc<R>();
        if constexpr (sizeof(R) == 4) {
          // complex64: two operand sets in rotation, so that the next chunk's
          // loads are in flight while a chunk is multiplied. Inside the loop
          // over chunk pairs the loads are unconditional (chunk indices
          // clamped; the last round's are never used) and scheduling barriers
          // keep their place, so that each product waits for its own operands
          // only. (The band is tile-aligned, so nch is a multiple of four; an
          // odd chunk would be taken after the loop.)
          trsm_ops<R, NCT> o0, o1;
          const int n2 = nch & ~1;
          if (n2 > 0) {
            trsm_load<R, NCT>(o0, Arow, N, X, nrhs, j0, nc, kc_of(0), lane);
            trsm_load<R, NCT>(o1, Arow, N, X, nrhs, j0, nc, kc_of(1), lane);
            for (int c = 0; c < n2; c += 2) {
              __builtin_amdgcn_sched_barrier(0);
              trsm_mul3<R, NCT>(o0, cre, cim, t3);
              __builtin_amdgcn_sched_barrier(0);
              trsm_load<R, NCT>(o0, Arow, N, X, nrhs, j0, nc, kc_of(min(c + 2, n2 - 2)), lane);
              __builtin_amdgcn_sched_barrier(0);
              trsm_mul3<R, NCT>(o1, cre, cim, t3);
              __builtin_amdgcn_sched_barrier(0);
              trsm_load<R, NCT>(o1, Arow, N, X, nrhs, j0, nc, kc_of(min(c + 3, n2 - 1)), lane);
            }
          }
          if (nch & 1) {
            trsm_load<R, NCT>(o0, Arow, N, X, nrhs, j0, nc, kc_of(nch - 1), lane);
            trsm_mul3<R, NCT>(o0, cre, cim, t3);
          }
        } else {
          trsm_ops<R, NCT> o0;
          for (int c = 0; c < nch; ++c) {
            trsm_load<R, NCT>(o0, Arow, N, X, nrhs, j0, nc, kc_of(c), lane);
            trsm_mul3<R, NCT>(o0, cre, cim, t3);
          }
        }
        // cre = sum a.re b.re, cim = sum a.im b.im, t3 = sum (a.re + a.im)(b.re + b.im)
#pragma unroll
        for (int rt = 0; rt < TRT; ++rt)
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) {
            const Acc t1 = cre[rt][ct], t2 = cim[rt][ct];
            cre[rt][ct] = t1 - t2;
            cim[rt][ct] = t3[rt][ct] - t1 - t2;
          }
      }
      // the super-block's own right-hand-side rows, all loaded before any is
      // used (columns beyond nc read the last column and are cleared by a
      // select): one memory round trip, where a guarded load per value had
      // compiled to a masked branch that waited for each load in turn
      C xv[TRT][NCT][4];
#pragma unroll
      for (int rt = 0; rt < TRT; ++rt)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * TRT * w + 16 * rt + acc_row<R>(lane, r);
            const int col = min(16 * ct + (lane & 15), nc - 1);
            xv[rt][ct][r] = X[(int64_t)(b0 + row) * nrhs + j0 + col];
          }
#pragma unroll
      for (int rt = 0; rt < TRT; ++rt)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * TRT * w + 16 * rt + acc_row<R>(lane, r);
            const int col = 16 * ct + (lane & 15);
            C x = col < nc ? xv[rt][ct][r] : czero<C>();
            x.x -= cre[rt][ct][r];
            x.y -= cim[rt][ct][r];
            Tb[row][col] = x;
          }
    }
    __syncthreads();
    // diagonal part: waves 0..3 hold the four 16-row tiles of a diagonal block
    const bool dw = w < NB / 16;
    for (int dq = 0; dq < nd; ++dq) {
      const int d = LOWER ? dq : nd - 1 - dq;
      const int db = b0 + NB * d;
      Acc yre[NCT], yim[NCT];
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) { yre[ct] = zacc<R>(); yim[ct] = zacc<R>(); }
      if (dw) {
        C dv[NB / 4];
#pragma unroll
        for (int kk = 0; kk < NB / 4; ++kk)
          dv[kk] = diag_inv_elem<R, LOWER>(A, N, db, 16 * w + (lane & 15), 4 * kk + (lane >> 4));
#pragma unroll
        for (int kk = 0; kk < NB / 4; ++kk)
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) {
            C bv = Tb[NB * d + 4 * kk + (lane >> 4)][16 * ct + (lane & 15)];
            cmfma<R>(dv[kk], bv, yre[ct], yim[ct]);
          }
      }
      __syncthreads();
      if (dw) {
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * w + acc_row<R>(lane, r);
            const int col = 16 * ct + (lane & 15);
            C v;
            v.x = yre[ct][r];
            v.y = yim[ct][r];
            Tb[NB * d + row][col] = v;
            if (col < nc) X[(int64_t)(db + row) * nrhs + j0 + col] = v;
          }
      }
      __syncthreads();
      // update the remaining diagonal blocks of this super-block, 16-row tiles
      const int nrem = LOWER ? (nd - 1 - d) : d;
      for (int t = w; t < 4 * nrem; t += TNW) {
        const int dd = LOWER ? d + 1 + t / 4 : t / 4;
        const int rt = t % 4;
        C av[NB / 4];
#pragma unroll
        for (int kk = 0; kk < NB / 4; ++kk)
          av[kk] = A[(int64_t)(b0 + NB * dd + 16 * rt + (lane & 15)) * N + db + 4 * kk + (lane >> 4)];
        Acc ure[NCT], uim[NCT];
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) { ure[ct] = zacc<R>(); uim[ct] = zacc<R>(); }
#pragma unroll
        for (int kk = 0; kk < NB / 4; ++kk)
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) {
            C bv = Tb[NB * d + 4 * kk + (lane >> 4)][16 * ct + (lane & 15)];
            cmfma<R>(av[kk], bv, ure[ct], uim[ct]);
          }
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = NB * dd + 16 * rt + acc_row<R>(lane, r);
            const int col = 16 * ct + (lane & 15);
            Tb[row][col].x -= ure[ct][r];
            Tb[row][col].y -= uim[ct][r];
          }
      }
      __syncthreads();
    }
  }
}

inline unsigned ceil_div(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

#define MX_TB(cls) \
  if (tm) tm->begin(cls)
#define MX_TE(cls) \
  if (tm) tm->end(cls)

template <typename R>
static void launch_panel(hipStream_t st, C_t<R>* pool, const int64_t* mat_off, const int32_t* Npad,
                         const int32_t* order, int32_t* piv, const int64_t* vec_off, int32_t* status, int32_t* pswap,
                         const int32_t* lim, int Nmax, int nact, int k0, int rows) {
  // rows of the panel that can be non-zero (structural bound from the host)
  const int m = std::min(Nmax - k0, rows);
  if (m <= PT * 1)
    hipLaunchKernelGGL((k_lu_panel<R, 1>), dim3(nact), dim3(PT), 0, st, pool, mat_off, Npad, order, piv, vec_off,
                       status, pswap, lim, k0);
  else if (m <= PT * 2)
    hipLaunchKernelGGL((k_lu_panel<R, 2>), dim3(nact), dim3(PT), 0, st, pool, mat_off, Npad, order, piv, vec_off,
                       status, pswap, lim, k0);
  else if (m <= PT * 4)
    hipLaunchKernelGGL((k_lu_panel<R, 4>), dim3(nact), dim3(PT), 0, st, pool, mat_off, Npad, order, piv, vec_off,
                       status, pswap, lim, k0);
  else
    hipLaunchKernelGGL((k_lu_panel<R, 8>), dim3(nact), dim3(PT), 0, st, pool, mat_off, Npad, order, piv, vec_off,
                       status, pswap, lim, k0);
}

// Batched LU with partial pivoting of all subdomain matrices (largest first,
// a subdomain drops out of a launch once its order is passed), then the
// inverses of the 64x64 diagonal blocks of U used by the triangular solves.
// Every trailing update visits only the tiles its band bookkeeping leaves
// (k_band_*), through a tile list walked by a fixed grid.
constexpr int UPDATE_GRID = 1024;   // workgroups of a tile-list update (2 per CU resident)

template <typename R>
void launch_lu(hipStream_t st, C_t<R>* pool, const int64_t* mat_off, const int32_t* Npad, const int32_t* order,
               int32_t* piv, const int64_t* vec_off, int32_t* status, int32_t* pswap,
               const std::vector<int32_t>& Nsorted, const LuBand& band, const std::vector<int32_t>& panel_rows,
               int group, KTimer* tm) {
  if (Nsorted.empty() || group < 1) return;
  const int Nmax = Nsorted[0];
  const int nsub = (int)Nsorted.size();
  auto active = [&](int k) {  // subdomains with N > k (Nsorted is descending)
    int a = 0;
    while (a < nsub && Nsorted[a] > k) ++a;
    return a;
  };
  const unsigned ctiles = ceil_div(Nmax, NB);
  const int np = band.np;
  hipLaunchKernelGGL(k_band_init, dim3(nsub), dim3(64), 0, st, nsub, Npad, np, band.ext_l, band.ext_u, band.work);
  // trailing update of the panels [pa, pb) over the tile box (rt0, ct0, mode)
  auto update = [&](int nact, int pa, int pb, int rt0, int ct0, int mode, int kl, int kd) {
    MX_TB(K_LU_UPDATE);
    hipLaunchKernelGGL(k_band_tiles, dim3(1), dim3(256), 0, st, nact, Npad, order, np, band.ext_l, band.ext_u, pa, pb,
                       rt0, ct0, mode, band.tptr, band.tbox, band.work, kd / NB);
    hipLaunchKernelGGL((k_lu_update_list<R>), dim3(UPDATE_GRID), dim3(256), 0, st, pool, mat_off, Npad, order, nact,
                       band.tptr, band.tbox, ct0, kl, kd);
    MX_TE(K_LU_UPDATE);
  };
  // Panels are taken in groups of `group`: the trailing matrix gets one
  // group*64-deep pass per group. Inside a group, panel i (i > 0) first
  // receives the group's earlier panels' update of its own column block
  // (rows below it), is factored, permutes the rows outside it, receives the
  // earlier panels' update of its own row block right of it, and then forms
  // its U12.
  for (int g0 = 0; g0 < Nmax; g0 += group * NB) {
    const int pa = g0 / NB;
    for (int i = 0; i < group; ++i) {
      const int ki = g0 + i * NB;
      if (ki >= Nmax) break;
      const int nact = active(ki);
      const int pk = ki / NB;
      if (i > 0) update(nact, pa, pk, pk, pk, 1, g0, i * NB);
      MX_TB(K_LU_PANEL);
      hipLaunchKernelGGL(k_band_limits, dim3(ceil_div(nact, 256)), dim3(256), 0, st, nact, Npad, order, np, band.band0,
                         band.ext_l, band.ext_u, band.lim, ki);
      launch_panel<R>(st, pool, mat_off, Npad, order, piv, vec_off, status, pswap, band.lim, Nmax, nact, ki,
                      pk < (int)panel_rows.size() ? panel_rows[pk] : Nmax - ki);
      hipLaunchKernelGGL((k_band_l<R>), dim3(nact), dim3(256), 0, st, pool, mat_off, Npad, order, piv, vec_off, np,
                         band.ext_l, band.lim, ki);
      MX_TE(K_LU_PANEL);
      MX_TB(K_LU_ROWPANEL);
      if (i > 0 && sizeof(R) == 4)  // complex64: the moved values fit in registers
        hipLaunchKernelGGL((k_lu_rowswap<R>), dim3(ctiles, nact), dim3(256), 0, st, pool, mat_off, Npad, order, pswap,
                           band.lim, ki);
      else
        hipLaunchKernelGGL((k_lu_rowpanel<R, MAXSW>), dim3(ctiles, nact), dim3(256), 0, st, pool, mat_off, Npad,
                           order, pswap, band.lim, ki, i == 0 ? 0 : 1);
      MX_TE(K_LU_ROWPANEL);
      const int kn = ki + NB;
      if (kn >= Nmax) continue;
      if (i > 0) {
        update(nact, pa, pk, pk, kn / NB, 2, g0, i * NB);
        MX_TB(K_LU_ROWPANEL);
        hipLaunchKernelGGL((k_lu_rowpanel<R, NB>), dim3(ctiles, nact), dim3(256), 0, st, pool, mat_off, Npad, order,
                           pswap, band.lim, ki, 2);
        MX_TE(K_LU_ROWPANEL);
      }
      MX_TB(K_LU_ROWPANEL);
      hipLaunchKernelGGL((k_band_u<R>), dim3(nact), dim3(256), 0, st, pool, mat_off, Npad, order, np, band.ext_u,
                         band.lim, ki);
      MX_TE(K_LU_ROWPANEL);
    }
    const int ke = g0 + group * NB;
    if (ke >= Nmax) break;
    update(active(ke), pa, pa + group, ke / NB, ke / NB, 0, g0, group * NB);
  }
  MX_TB(K_LU_INV);
  hipLaunchKernelGGL((k_inv_upper<R>), dim3(ceil_div(Nmax, NB), (unsigned)Nsorted.size()), dim3(256), 0, st, pool,
                     mat_off, Npad, order);
  MX_TE(K_LU_INV);
}
template void launch_lu<float>(hipStream_t, float2*, const int64_t*, const int32_t*, const int32_t*, int32_t*,
                               const int64_t*, int32_t*, int32_t*, const std::vector<int32_t>&, const LuBand&,
                               const std::vector<int32_t>&, int, KTimer*);
template void launch_lu<double>(hipStream_t, double2*, const int64_t*, const int32_t*, const int32_t*, int32_t*,
                                const int64_t*, int32_t*, int32_t*, const std::vector<int32_t>&, const LuBand&,
                                const std::vector<int32_t>&, int, KTimer*);

void launch_perm(hipStream_t st, int32_t nsub, const int32_t* Npad, const int64_t* vec_off, const int32_t* dense_edge,
                 const int32_t* piv, int32_t* perm_scratch, int32_t* rowsrc) {
  if (nsub > 0)
    hipLaunchKernelGGL(k_perm, dim3(nsub), dim3(64), 0, st, nsub, Npad, vec_off, dense_edge, piv, perm_scratch,
                       rowsrc);
}

template <typename R>
void launch_trsm(hipStream_t st, const C_t<R>* pool, const int64_t* mat_off, const int32_t* Npad,
                 const int64_t* vec_off, const int32_t* order, C_t<R>* xloc, int nsub, int nrhs,
                 const int32_t* trs_lo, const int32_t* trs_hi, int np, int cols, KTimer* tm) {
  if (nsub <= 0 || nrhs <= 0) return;
  const dim3 block(64 * trsm_waves<R>());
  if (cols == 16) {
    const dim3 grid(nsub, ceil_div(nrhs, 16));
    MX_TB(K_TRSM_LOWER);
    hipLaunchKernelGGL((k_trsm<R, true, 1>), grid, block, 0, st, pool, mat_off, Npad, vec_off, order, xloc, nrhs,
                       trs_lo, trs_hi, np);
    MX_TE(K_TRSM_LOWER);
    MX_TB(K_TRSM_UPPER);
    hipLaunchKernelGGL((k_trsm<R, false, 1>), grid, block, 0, st, pool, mat_off, Npad, vec_off, order, xloc, nrhs,
                       trs_lo, trs_hi, np);
    MX_TE(K_TRSM_UPPER);
  } else {
    const dim3 grid(nsub, ceil_div(nrhs, 32));
    MX_TB(K_TRSM_LOWER);
    hipLaunchKernelGGL((k_trsm<R, true, 2>), grid, block, 0, st, pool, mat_off, Npad, vec_off, order, xloc, nrhs,
                       trs_lo, trs_hi, np);
    MX_TE(K_TRSM_LOWER);
    MX_TB(K_TRSM_UPPER);
    hipLaunchKernelGGL((k_trsm<R, false, 2>), grid, block, 0, st, pool, mat_off, Npad, vec_off, order, xloc, nrhs,
                       trs_lo, trs_hi, np);
    MX_TE(K_TRSM_UPPER);
  }
}
template void launch_trsm<float>(hipStream_t, const float2*, const int64_t*, const int32_t*, const int64_t*,
                                 const int32_t*, float2*, int, int, const int32_t*, const int32_t*, int, int,
                                 KTimer*);
template void launch_trsm<double>(hipStream_t, const double2*, const int64_t*, const int32_t*, const int64_t*,
                                  const int32_t*, double2*, int, int, const int32_t*, const int32_t*, int, int,
                                  KTimer*);

int lu_max_swap_rows() { return MAXSW; }

}  // namespace mx
