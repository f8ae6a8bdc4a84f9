// Tall-skinny complex128 products of block FGMRES (block Gram-Schmidt, QR of
// a block through its Gram matrix, solution update). Blocks are row-major
// [rows][ld] device arrays: row r of a block of s columns holds its s
// complex values contiguously, as the right-hand-side blocks of the solver.
//
//   k_bdot_* P[chunk] = A[chunk rows, 0:ka]^H B[chunk rows, 0:s]   (partials;
//            _mfma for ka > 32, _narrow for ka <= 32)
//   k_bsum   out = sum over chunks of P (fixed order: deterministic)
//   k_bupd   Wout = beta Win + alpha A[:, 0:ka] H (H ka x s; Win may be Wout:
//            each output element is read and written by one lane)
//   k_bcopy  dst[:, 0:s] = src[:, 0:s] between blocks of different ld
//
// All products run on the FP64 matrix cores (16x16x4 MFMA, complex products in
// the 3-multiplication form, operands straight from memory).
#include "mx_device.h"
#include "mx_kernels.h"

namespace mx {

namespace {
constexpr int BT = 256;   // threads per workgroup
constexpr int BA = 128;   // columns of A per k_bdot_mfma workgroup
constexpr int BR = 32;    // row-chunk granularity of the block dots
constexpr int UR = 128;   // rows per k_bupd_mfma workgroup
constexpr int UA = 64;    // rows of H per LDS stage of k_bupd_mfma (32 KB)
}  // namespace

// The same partial products on the FP64 matrix cores, for ka > 32: a
// workgroup takes a 128-wide tile of A's columns (wave w: columns 32w..32w+31
// as two 16-wide MFMA tiles) and all 32 columns of B (two tiles), and walks
// the rows of its chunk 4 at a time (the MFMA depth); lane l holds row
// 4c + (l >> 4) of column l & 15 of each tile, loaded straight from memory.
// Capped at 170 registers, the accumulators move out of the AGPRs and the
// kernel fits in 128, four waves per SIMD (two at the default allocation).
__global__ void __launch_bounds__(BT, 3) k_bdot_mfma(int64_t nrows, int64_t rows_per_chunk, int ka, int s,
                                                  const double2* __restrict__ A, int64_t lda,
                                                  const double2* __restrict__ B, int64_t ldb,
                                                  double2* __restrict__ P) {
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_chunk;
  const int64_t r1 = min(nrows, r0 + rows_per_chunk);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int abase = blockIdx.y * BA + 32 * w;
  if (abase >= ka) return;  // whole wave idle (no barriers in this kernel)
  const int kq = lane >> 4, cl = lane & 15;
  // 3-multiplication form: t1 = sum ar br, t2 = sum ai bi,
  // t3 = sum (ar - ai)(br + bi); conj(a) b = (t1 + t2, t3 - t1 + t2)
  Acc_t<double> t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) t1[t][u][q] = t2[t][u][q] = t3[t][u][q] = 0.0;
  const bool aok0 = abase + cl < ka, aok1 = abase + 16 + cl < ka;
  const bool bok0 = cl < s, bok1 = 16 + cl < s;
  // every load unconditional, from a clamped (valid) row and column, with the
  // values outside the product cleared afterwards by selects; two operand
  // sets in rotation (no register copies, which would wait for the loads):
  // each group of 4 rows is loaded while the previous one is multiplied, so
  // each wave keeps two groups' loads in flight. A group past the chunk's end
  // contributes exact zeros.
  const double2* Ap0 = A + min(abase + cl, ka - 1);
  const double2* Ap1 = A + min(abase + 16 + cl, ka - 1);
  const double2* Bp0 = B + min(cl, s - 1);
  const double2* Bp1 = B + min(16 + cl, s - 1);
  const double2 z2 = make_double2(0.0, 0.0);
  auto load = [&](int64_t rs, double2 (&a)[2], double2 (&b)[2]) {
    const int64_t r = min(rs + kq, r1 - 1);
    a[0] = Ap0[r * lda];
    a[1] = Ap1[r * lda];
    b[0] = Bp0[r * ldb];
    b[1] = Bp1[r * ldb];
  };
  auto multiply = [&](int64_t rs, const double2 (&a)[2], const double2 (&b)[2]) {
    const bool rok = rs + kq < r1;
    const double2 ac[2] = {rok && aok0 ? a[0] : z2, rok && aok1 ? a[1] : z2};
    const double2 bc[2] = {rok && bok0 ? b[0] : z2, rok && bok1 ? b[1] : z2};
    const double ad[2] = {ac[0].x - ac[0].y, ac[1].x - ac[1].y};
    const double bs[2] = {bc[0].x + bc[0].y, bc[1].x + bc[1].y};
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        t1[t][u] = mfma(ac[t].x, bc[u].x, t1[t][u]);
        t2[t][u] = mfma(ac[t].y, bc[u].y, t2[t][u]);
        t3[t][u] = mfma(ad[t], bs[u], t3[t][u]);
      }
  };
  if (r0 < r1) {
    double2 a0[2], b0[2], a1[2], b1[2];
    load(r0, a0, b0);
    for (int64_t rs = r0; rs < r1; rs += 8) {
      load(rs + 4, a1, b1);
      __builtin_amdgcn_sched_barrier(0);
      multiply(rs, a0, b0);
      __builtin_amdgcn_sched_barrier(0);
      load(rs + 8, a0, b0);
      __builtin_amdgcn_sched_barrier(0);
      multiply(rs + 4, a1, b1);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  double2* out = P + (int64_t)blockIdx.x * ka * s;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int a = abase + 16 * t + acc_row<double>(lane, q);
        const int b = 16 * u + cl;
        if (a < ka && b < s)
          out[(int64_t)a * s + b] =
              make_double2(t1[t][u][q] + t2[t][u][q], t3[t][u][q] - t1[t][u][q] + t2[t][u][q]);
      }
}

// The narrow products (ka <= 32, e.g. Gram matrices) on the FP64 matrix
// cores: every wave computes the whole 32 x 32 output over every fourth group
// of 4 rows of the chunk, and the four waves' sums are added in a fixed order
// through LDS before the chunk's partial is written. 32 KB of LDS and the
// occupancy bound keep the accumulators in ordinary registers (with 64 KB and
// no bound the compiler held them in the accumulation registers and copied
// all 96 of them out and back on every step of the loop).
__global__ void __launch_bounds__(BT, 4) k_bdot_narrow(int64_t nrows, int64_t rows_per_chunk, int ka, int s,
                                                    const double2* __restrict__ A, int64_t lda,
                                                    const double2* __restrict__ B, int64_t ldb,
                                                    double2* __restrict__ P) {
  __shared__ double2 red[2][32][32];
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_chunk;
  const int64_t r1 = min(nrows, r0 + rows_per_chunk);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int kq = lane >> 4, cl = lane & 15;
  Acc_t<double> t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) t1[t][u][q] = t2[t][u][q] = t3[t][u][q] = 0.0;
  const bool aok0 = cl < ka, aok1 = 16 + cl < ka;
  const bool bok0 = cl < s, bok1 = 16 + cl < s;
  for (int64_t rs = r0 + 4 * w; rs < r1; rs += 16) {
    const int64_t r = rs + kq;
    const bool rok = r < r1;
    double2 av[2], bv[2];
    av[0] = rok && aok0 ? A[r * lda + cl] : make_double2(0.0, 0.0);
    av[1] = rok && aok1 ? A[r * lda + 16 + cl] : make_double2(0.0, 0.0);
    bv[0] = rok && bok0 ? B[r * ldb + cl] : make_double2(0.0, 0.0);
    bv[1] = rok && bok1 ? B[r * ldb + 16 + cl] : make_double2(0.0, 0.0);
    const double ad[2] = {av[0].x - av[0].y, av[1].x - av[1].y};
    const double bs[2] = {bv[0].x + bv[0].y, bv[1].x + bv[1].y};
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        t1[t][u] = mfma(av[t].x, bv[u].x, t1[t][u]);
        t2[t][u] = mfma(av[t].y, bv[u].y, t2[t][u]);
        t3[t][u] = mfma(ad[t], bs[u], t3[t][u]);
      }
  }
  // the four waves' sums added in a fixed order through one 32 KB array:
  // (w0 + w2) + (w1 + w3)
  if (w >= 2) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          red[w - 2][16 * t + acc_row<double>(lane, q)][16 * u + cl] =
              make_double2(t1[t][u][q] + t2[t][u][q], t3[t][u][q] - t1[t][u][q] + t2[t][u][q]);
  }
  __syncthreads();
  if (w < 2) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          double2& e = red[w][16 * t + acc_row<double>(lane, q)][16 * u + cl];
          const double2 o = e;
          e = make_double2(t1[t][u][q] + t2[t][u][q] + o.x, t3[t][u][q] - t1[t][u][q] + t2[t][u][q] + o.y);
        }
  }
  __syncthreads();
  double2* out = P + (int64_t)blockIdx.x * ka * s;
  for (int e = threadIdx.x; e < 32 * 32; e += BT) {
    const int a = e / 32, b = e % 32;
    if (a >= ka || b >= s) continue;
    out[(int64_t)a * s + b] = make_double2(red[0][a][b].x + red[1][a][b].x, red[0][a][b].y + red[1][a][b].y);
  }
}

// Wout = beta Win + alpha A H (also written to Wout2 when given) on the FP64
// matrix cores: a workgroup takes 128
// rows (wave w: rows 32w..32w+31 as two 16-row MFMA tiles) and all 32
// columns; H is staged through LDS 64 rows at a time (32 KB, so that LDS
// admits four workgroups per CU, the register cap's occupancy: four waves per
// SIMD, with two values spilled outside the loops); lane l holds A's row
// l & 15 of each tile at column 4c + (l >> 4).
__global__ void __launch_bounds__(BT, 3) k_bupd_mfma(int64_t nrows, int ka, int s, const double2* __restrict__ A,
                                                  int64_t lda, const double2* __restrict__ H,
                                                  const double2* Win, int64_t ldwin, double2* Wout,
                                                  int64_t ldwout, double alpha, double beta, double2* Wout2,
                                                  int64_t ldwout2) {
  __shared__ double2 Hs[UA][32];
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int kq = lane >> 4, cl = lane & 15;
  const int64_t rw = (int64_t)blockIdx.x * UR + 32 * w;
  // 3-multiplication form: t1 = sum ar hr, t2 = sum ai hi,
  // t3 = sum (ar + ai)(hr + hi); a h = (t1 - t2, t3 - t1 - t2)
  Acc_t<double> t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) t1[t][u][q] = t2[t][u][q] = t3[t][u][q] = 0.0;
  const bool rok0 = rw + cl < nrows, rok1 = rw + 16 + cl < nrows;
  // A's loads unconditional from clamped (valid) rows and columns, cleared
  // afterwards by selects; two operand sets in rotation, so that each group
  // of 4 columns is loaded while the previous one is multiplied
  const double2* A0 = A + min(rw + cl, nrows - 1) * lda;
  const double2* A1 = A + min(rw + 16 + cl, nrows - 1) * lda;
  const double2 z2 = make_double2(0.0, 0.0);
  auto load = [&](int a, double2 (&av)[2]) {
    const int ac = min(a + kq, ka - 1);
    av[0] = A0[ac];
    av[1] = A1[ac];
  };
  auto multiply = [&](int aa, int na, const double2 (&av)[2]) {
    const bool aok = aa + kq < na;
    const double2 ac[2] = {rok0 && aok ? av[0] : z2, rok1 && aok ? av[1] : z2};
    const int ah = min(aa + kq, UA - 1);
    const double2 hv[2] = {Hs[ah][cl], Hs[ah][16 + cl]};
    const double as[2] = {ac[0].x + ac[0].y, ac[1].x + ac[1].y};
    const double hs[2] = {hv[0].x + hv[0].y, hv[1].x + hv[1].y};
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        t1[t][u] = mfma(ac[t].x, hv[u].x, t1[t][u]);
        t2[t][u] = mfma(ac[t].y, hv[u].y, t2[t][u]);
        t3[t][u] = mfma(as[t], hs[u], t3[t][u]);
      }
  };
  for (int a0 = 0; a0 < ka; a0 += UA) {
    const int na = min(UA, ka - a0);
    __syncthreads();
    for (int e = tid; e < UA * 32; e += BT) {
      const int aa = e / 32, bb = e % 32;
      Hs[aa][bb] = (aa < na && bb < s) ? H[(int64_t)(a0 + aa) * s + bb] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    double2 x0[2], x1[2];
    load(a0, x0);
    for (int aa = 0; aa < na; aa += 8) {
      load(a0 + aa + 4, x1);
      __builtin_amdgcn_sched_barrier(0);
      multiply(aa, na, x0);
      __builtin_amdgcn_sched_barrier(0);
      load(a0 + aa + 8, x0);
      __builtin_amdgcn_sched_barrier(0);
      multiply(aa + 4, na, x1);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // epilogue per 16-row tile: the 8 values of Win it needs are loaded
  // together (clamped, valid addresses) before any is used, one memory round
  // trip instead of eight; each element is read and written by one lane, so
  // Win may be Wout
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    double2 wv[2][4];
    if (beta != 0.0) {
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t r = min(rw + 16 * t + acc_row<double>(lane, q), nrows - 1);
          wv[u][q] = Win[r * ldwin + min(16 * u + cl, s - 1)];
        }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = rw + 16 * t + acc_row<double>(lane, q);
        const int b = 16 * u + cl;
        if (r >= nrows || b >= s) continue;
        double re = alpha * (t1[t][u][q] - t2[t][u][q]);
        double im = alpha * (t3[t][u][q] - t1[t][u][q] - t2[t][u][q]);
        if (beta != 0.0) {
          re = fma(beta, wv[u][q].x, re);
          im = fma(beta, wv[u][q].y, im);
        }
        Wout[r * ldwout + b] = make_double2(re, im);
        if (Wout2) Wout2[r * ldwout2 + b] = make_double2(re, im);
      }
  }
}

// out[i] = sum over chunks c of P[c][i], i < n; a workgroup takes 32
// consecutive outputs, its 8 thread groups every 8th chunk, and the 8
// partial sums are added in group order (the same order on every run)
__global__ void __launch_bounds__(BT) k_bsum(int nchunks, int64_t n, const double2* __restrict__ P,
                                             double2* __restrict__ out) {
  __shared__ double2 part[8][32];
  const int lane = threadIdx.x & 31, grp = threadIdx.x >> 5;
  const int64_t i = (int64_t)blockIdx.x * 32 + lane;
  double re = 0, im = 0;
  if (i < n)
    for (int c = grp; c < nchunks; c += 8) {
      const double2 v = P[(int64_t)c * n + i];
      re += v.x;
      im += v.y;
    }
  part[grp][lane] = make_double2(re, im);
  __syncthreads();
  if (grp == 0 && i < n) {
    double sr = 0, si = 0;
    for (int g = 0; g < 8; ++g) {
      sr += part[g][lane].x;
      si += part[g][lane].y;
    }
    out[i] = make_double2(sr, si);
  }
}

__global__ void k_bcopy(int64_t nrows, int s, const double2* __restrict__ src, int64_t lds, double2* __restrict__ dst,
                        int64_t ldd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows * s) return;
  const int64_t r = i / s;
  const int b = (int)(i % s);
  dst[r * ldd + b] = src[r * lds + b];
}

int block_chunks(int64_t nrows, int ka, int64_t* rows_per_chunk) {
  const int ntile = ka <= 32 ? 1 : (ka + BA - 1) / BA;
  int64_t want = ka <= 32 ? 512 : std::max<int64_t>(64, std::min<int64_t>(1024, 2048 / ntile));
  int64_t rpc = (nrows + want - 1) / want;
  rpc = std::max<int64_t>(BR, (rpc + BR - 1) / BR * BR);
  *rows_per_chunk = rpc;
  return (int)((nrows + rpc - 1) / rpc);
}

// entries of the partial-product buffer launch_bdot needs for ka <= ka_max
int64_t block_partial_max(int ka_max, int s) { return std::max<int64_t>((int64_t)2048 * BA, (int64_t)64 * ka_max) * s; }

void launch_bdot(hipStream_t st, int64_t nrows, int ka, int s, const double2* A, int64_t lda, const double2* B,
                 int64_t ldb, double2* P, double2* out) {
  if (nrows <= 0 || ka <= 0 || s <= 0) return;
  int64_t rpc;
  const int nch = block_chunks(nrows, ka, &rpc);
  if (ka <= 32)
    hipLaunchKernelGGL(k_bdot_narrow, dim3(nch, 1), dim3(BT), 0, st, nrows, rpc, ka, s, A, lda, B, ldb, P);
  else
    hipLaunchKernelGGL(k_bdot_mfma, dim3(nch, (ka + BA - 1) / BA), dim3(BT), 0, st, nrows, rpc, ka, s, A, lda, B,
                       ldb, P);
  const int64_t n = (int64_t)ka * s;
  hipLaunchKernelGGL(k_bsum, dim3((unsigned)((n + 31) / 32)), dim3(BT), 0, st, nch, n, P, out);
}

void launch_bupd(hipStream_t st, int64_t nrows, int ka, int s, const double2* A, int64_t lda, const double2* H,
                 const double2* Win, int64_t ldwin, double2* Wout, int64_t ldwout, double alpha, double beta,
                 double2* Wout2, int64_t ldwout2) {
  if (nrows <= 0 || s <= 0) return;
  hipLaunchKernelGGL(k_bupd_mfma, dim3((unsigned)((nrows + UR - 1) / UR)), dim3(BT), 0, st, nrows, ka, s, A, lda, H,
                     Win, ldwin, Wout, ldwout, alpha, beta, Wout2, ldwout2);
}

void launch_bcopy(hipStream_t st, int64_t nrows, int s, const double2* src, int64_t lds, double2* dst, int64_t ldd) {
  const int64_t n = nrows * s;
  if (n > 0) hipLaunchKernelGGL(k_bcopy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, nrows, s, src, lds, dst, ldd);
}

}  // namespace mx
