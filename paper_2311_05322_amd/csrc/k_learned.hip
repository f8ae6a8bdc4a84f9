// Learned coarse-space correction: per-subdomain 4x4x4 lattice prolongation,
// pooling of block vectors onto the lattice, the per-subdomain network
// (4-layer MLP + 2 message-passing layers) and its training kernels.
//
// Network arithmetic: the operands of every matrix product are rounded to
// bfloat16 (round to nearest even) as they are staged into LDS and multiplied
// on the 16x16x32 bf16 matrix cores with FP32 accumulation; biases, GELU, the
// loss and the Adam update run in FP32 on FP32 master weights.
#include "mx_device.h"
#include "mx_kernels.h"

namespace mx {

namespace {

constexpr int NCO = 192;   // complex lattice coefficients (64 nodes x 3 components)
constexpr int NIN = 384;   // real channels [Re | Im]

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

__device__ inline float gelu_f(float z) {
  const float a = 0.7978845608028654f;
  return 0.5f * z * (1.f + tanhf(a * (z + 0.044715f * z * z * z)));
}
__device__ inline float gelu_grad_f(float z) {
  const float a = 0.7978845608028654f;
  float t = tanhf(a * (z + 0.044715f * z * z * z));
  return 0.5f * (1.f + t) + 0.5f * z * (1.f - t * t) * a * (1.f + 3.f * 0.044715f * z * z);
}

// P[row][3 node + k] = sum_q w_q phi_node(x_a + s_q t) t_k  (3-point Gauss)
__global__ void k_coarse_P(int64_t nrows, const int32_t* __restrict__ row_sub, const int32_t* __restrict__ dofs,
                           const int32_t* __restrict__ edges, const double* __restrict__ xyz,
                           const double* __restrict__ box, float* __restrict__ P) {
  int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (row >= nrows) return;
  const int s = row_sub[row];
  const int e = dofs[row];
  double xa[3], t[3], lo[3], span[3];
  for (int c = 0; c < 3; ++c) {
    xa[c] = xyz[3 * (size_t)edges[2 * (size_t)e] + c];
    t[c] = xyz[3 * (size_t)edges[2 * (size_t)e + 1] + c] - xa[c];
    lo[c] = box[6 * (size_t)s + c];
    span[c] = (box[6 * (size_t)s + 3 + c] - lo[c]) / 3.0;
  }
  float* pr = P + row * NCO;
  for (int k = 0; k < NCO; ++k) pr[k] = 0.f;
  const double sq[3] = {0.1127016653792583, 0.5, 0.8872983346207417};
  const double wq[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
  for (int q = 0; q < 3; ++q) {
    double psi[3][4];
    for (int c = 0; c < 3; ++c) {
      double xi = (xa[c] + sq[q] * t[c] - lo[c]) / span[c];
      for (int a = 0; a < 4; ++a) psi[c][a] = fmax(0.0, 1.0 - fabs(xi - a));
    }
    for (int cz = 0; cz < 4; ++cz) {
      if (psi[2][cz] == 0.0) continue;
      for (int by = 0; by < 4; ++by) {
        if (psi[1][by] == 0.0) continue;
        for (int ax = 0; ax < 4; ++ax) {
          double phi = psi[0][ax] * psi[1][by] * psi[2][cz];
          if (phi == 0.0) continue;
          const int node = ax + 4 * by + 16 * cz;
          for (int k = 0; k < 3; ++k) pr[3 * node + k] += (float)(wq[q] * phi * t[k]);
        }
      }
    }
  }
}

// X[(j*nsub + i)][k] (+192 for Im) = sum_l w_l P[l][k] v[dofs[l]][j] / s_j for the
// right-hand sides j0 .. j0+nj-1 (nj <= 32); w = D weights or 1.
// Two kernels: k_pool_part splits each subdomain's rows into PS slices, one
// workgroup per (subdomain, slice), and writes the slice's sums; k_pool_sum
// adds the slices in a fixed order and scales (so the result does not depend
// on scheduling). k_pool_part forms the slice's (192 coefficients) x (64 =
// 32 right-hand sides x [re, im]) product P^T V on the FP32 matrix cores,
// 4 rows per step: wave w holds the coefficient tiles 3w .. 3w+2 against all
// four column tiles; P rows (times the optional weight) and V rows (cast to
// FP32, column n = 2 j + [re, im]) go straight into MFMA operands. Every
// load of a step is unconditional (rows past the slice read row r0, columns
// past nj column j0) and the unused values are cleared by bit masks: with
// selects the compiler moved each V load into its own masked branch that
// waited for it, five dependent memory round trips per step.
constexpr int PS = 8;
template <bool WEIGHTED>
__global__ void __launch_bounds__(256, 5) k_pool_part(int nsub, const int64_t* __restrict__ dof_ptr,
                                                   const int32_t* __restrict__ dofs, const float* __restrict__ P,
                                                   const double* __restrict__ wts, const double2* __restrict__ v,
                                                   int nrhs, int j0, int nj, float* __restrict__ Xp) {
  const int i = blockIdx.x, y = blockIdx.y;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  f32x4 acc[3][4];
#pragma unroll
  for (int mt = 0; mt < 3; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t a0 = dof_ptr[i], a1 = dof_ptr[i + 1];
  const int64_t len = (a1 - a0 + PS - 1) / PS;
  const int64_t r0 = a0 + y * len, r1 = min(a1, r0 + len);
  // the slice's DOF indices (at most 8192 / PS rows: subdomains hold at most
  // 8192 unknowns) staged in LDS, so that a step's V loads wait on an LDS
  // read instead of a dependent global load
  __shared__ int32_t sdof[8192 / PS];
  for (int64_t r = r0 + tid; r < r1; r += 256) sdof[r - r0] = dofs[r];
  __syncthreads();
  // B operand columns of this lane: n = 16 nt + lane % 16 -> j = n / 2, part n % 2
  int jb[4];
  uint32_t bmask[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int n = 16 * nt + (lane & 15);
    const bool bok = (n >> 1) < nj;
    jb[nt] = bok ? n >> 1 : 0;
    bmask[nt] = bok ? 0xffffffffu : 0u;
  }
  const int part = lane & 1;
  for (int64_t kr = r0; kr < r1; kr += 4) {
    // A[m][k] = P[row k][coef m], B[k][n] = w_row V[row k][n], k = lane / 16
    const int64_t row = kr + (lane >> 4);
    const bool ok = row < r1;
    const int64_t rr = ok ? row : r0;
    const uint32_t rmask = ok ? 0xffffffffu : 0u;
    float a[3], b[4];
    double d[4];
#pragma unroll
    for (int mt = 0; mt < 3; ++mt) a[mt] = P[rr * NCO + 16 * (3 * w + mt) + (lane & 15)];
    const double* vr = reinterpret_cast<const double*>(v + (int64_t)sdof[rr - r0] * nrhs + j0) + part;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) d[nt] = vr[2 * jb[nt]];
    const float wr = WEIGHTED ? (float)wts[rr] : 1.f;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
      b[nt] = __uint_as_float(__float_as_uint(wr * (float)d[nt]) & (bmask[nt] & rmask));
#pragma unroll
    for (int mt = 0; mt < 3; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = mfma(a[mt], b[nt], acc[mt][nt]);
  }
  // acc[mt][nt][r]: coefficient 16 (3w + mt) + 4 (lane / 16) + r, column 16 nt + lane % 16; every slice
  // writes all 32 right-hand sides (those beyond nj hold zeros)
  float* xp = Xp + (int64_t)y * 32 * nsub * NIN;
#pragma unroll
  for (int mt = 0; mt < 3; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int coef = 16 * (3 * w + mt) + acc_row<float>(lane, r);
        xp[((int64_t)((16 * nt + (lane & 15)) >> 1) * nsub + i) * NIN + part * NCO + coef] = acc[mt][nt][r];
      }
}

// X[(j0 + jj) * nsub + i][k] = (sum over slices y in order of Xp[y][jj * nsub + i][k]) / s_(j0+jj)
__global__ void __launch_bounds__(256) k_pool_sum(int nsub, int j0, int nj, const double* __restrict__ scale,
                                                  const float* __restrict__ Xp, float* __restrict__ X,
                                                  int64_t xrows_stride) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)nj * nsub * NIN) return;
  const int64_t row = e / NIN;
  const int k = (int)(e % NIN);
  const int jj = (int)(row / nsub), i = (int)(row % nsub);
  float sum = 0.f;
  for (int y = 0; y < PS; ++y) sum += Xp[((int64_t)y * 32 * nsub + row) * NIN + k];
  const double sj = scale[j0 + jj];
  const float inv = sj > 0 ? (float)(1.0 / sj) : 0.f;
  X[((int64_t)(j0 + jj) * nsub + i) * xrows_stride + k] = sum * inv;
}

// xloc[vec_off[i] + lpos[l]][j] += alpha * s_j * sum_k P[l][k] (c_re[k] + j c_im[k])
// (lpos: dense row of the subdomain DOF row l). On the FP32 matrix cores:
// per 16-row block of the subdomain, (16 rows x 192) P times (192 x 64)
// coefficients, column n = 2 j + [re, im]; the coefficients of the block of
// right-hand sides (scaled by alpha s_j) are staged in LDS as [k][n]; each
// wave takes every fourth 16-row block of its workgroup's share.
template <typename C>
__global__ void __launch_bounds__(256, 3) k_coarse_apply(const int32_t* __restrict__ lpos,
                                                      const int64_t* __restrict__ dof_ptr,
                                                      const int64_t* __restrict__ vec_off, const float* __restrict__ P,
                                                      const float* __restrict__ Cn, int nsub, int nrhs, int j0, int nj,
                                                      const double* __restrict__ scale, float alpha,
                                                      C* __restrict__ xloc) {
  typedef decltype(C().x) R;
  __shared__ float Cs[NCO][64];
  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  for (int e = tid; e < NCO * 64; e += 256) {
    const int k = e >> 6, n = e & 63, jj = n >> 1;
    float c = 0.f;
    if (jj < nj) c = alpha * (float)scale[j0 + jj] * Cn[((int64_t)(j0 + jj) * nsub + i) * NIN + (n & 1) * NCO + k];
    Cs[k][n] = c;
  }
  __syncthreads();
  const int64_t r0 = dof_ptr[i], r1 = dof_ptr[i + 1];
  const int64_t voff = vec_off[i];
  const int64_t step = 16 * 4 * (int64_t)gridDim.y;
  for (int64_t rb = r0 + 16 * ((int64_t)blockIdx.y * 4 + w); rb < r1; rb += step) {
    // A[m][k] = P[row rb + m][k] (rows past the end read the last row; not
    // written). K is taken in blocks of 64 with lane group g = lane / 16
    // holding k = 64 kb + 16 g + t at step t, so that a lane reads its 16
    // coefficients of a block as four 16-byte loads; all twelve are issued
    // before the first product.
    const float4* pr = reinterpret_cast<const float4*>(P + min(rb + (lane & 15), r1 - 1) * NCO) + 4 * (lane >> 4);
    float4 p4[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) p4[q] = pr[16 * (q >> 2) + (q & 3)];
    // destination rows of this lane's results (clamped, so that every load
    // below is in bounds; only rows < r1 are written)
    int64_t xoff[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = rb + acc_row<float>(lane, r);
      xoff[r] = (voff + lpos[row < r1 ? row : r1 - 1]) * nrhs + j0;
    }
    f32x4 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < NCO / 64; ++kb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 t4 = p4[4 * kb + q];
        const float a[4] = {t4.x, t4.y, t4.z, t4.w};
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int nt = 0; nt < 4; ++nt)
            acc[nt] = mfma(a[e], Cs[64 * kb + 16 * (lane >> 4) + 4 * q + e][16 * nt + (lane & 15)], acc[nt]);
        // keep the scheduler from hoisting every LDS operand of the 192
        // products at once (their registers would spill)
        __builtin_amdgcn_sched_barrier(0);
      }
    // acc[nt][r]: row rb + 4 (lane / 16) + r, column 16 nt + lane % 16 -> j, part.
    // Read-modify-write of xloc with every load issued before the first
    // store (a load after a store to the same array would wait for it).
    R xv[4][4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int n = 16 * nt + (lane & 15), jj = n >> 1;
      const int jc = jj < nj ? jj : 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) xv[nt][r] = reinterpret_cast<const R*>(xloc + xoff[r] + jc)[n & 1];
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int n = 16 * nt + (lane & 15), jj = n >> 1;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = rb + acc_row<float>(lane, r);
        if (jj < nj && row < r1) reinterpret_cast<R*>(xloc + xoff[r] + jj)[n & 1] = xv[nt][r] + (R)acc[nt][r];
      }
    }
  }
}

// G-apply: out[(j*nsub+i)][0:384] = G_i (in[(j*nsub+i)][0:192] , [192:384]) (real G on Re and Im)
__global__ void __launch_bounds__(192) k_gapply(int nsub, int nrhs, const double* __restrict__ G,
                                                const float* __restrict__ in, float* __restrict__ out) {
  const int i = blockIdx.x, j = blockIdx.y, k = threadIdx.x;
  const double* g = G + (int64_t)i * NCO * NCO + (int64_t)k * NCO;
  const float* x = in + ((int64_t)j * nsub + i) * NIN;
  double re = 0, im = 0;
  for (int m = 0; m < NCO; ++m) {
    re += g[m] * x[m];
    im += g[m] * x[NCO + m];
  }
  float* y = out + ((int64_t)j * nsub + i) * NIN;
  y[k] = (float)re;
  y[NCO + k] = (float)im;
}

// PDP_i = P_i^T diag(D_i) P_i  (192 x 192 per subdomain, FP64 accumulation)
__global__ void __launch_bounds__(192) k_pdp(const int64_t* __restrict__ dof_ptr, const float* __restrict__ P,
                                             const double* __restrict__ D, double* __restrict__ out) {
  const int i = blockIdx.x, a = blockIdx.y, b = threadIdx.x;
  double acc = 0;
  for (int64_t l = dof_ptr[i]; l < dof_ptr[i + 1]; ++l) acc += D[l] * (double)P[l * NCO + a] * (double)P[l * NCO + b];
  out[((int64_t)i * NCO + a) * NCO + b] = acc;
}

// ---------------------------------------------------------------------------
// GEMM: C[m][n] (= or +=) sum_k a(m,k) b(k,n) (+ bias[n]), optional GELU with
// the pre-activation kept in Z; a(m,k) = TA ? A[k*lda+m] : A[m*lda+k],
// b(k,n) = TB ? B[n*ldb+k] : B[k*ldb+n].  Operands rounded to bfloat16
// (round to nearest even) as they are staged into LDS, products on the bf16
// matrix cores (16x16x32, FP32 accumulation: a bf16 x bf16 product is exact
// in FP32, so the result differs from FP32 arithmetic on the rounded operands
// only in the order of the additions). 64x64 tiles, 32-deep K chunks, both
// operands stored k-contiguous in LDS so that a lane's eight k values are
// one 16-byte read; 4 waves x (2x2) MFMA tiles. gridDim.z > 1 splits K; each
// split writes its own slice C + z*M*ldc.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

__device__ inline unsigned short bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u)  // inf stays inf, a NaN stays a NaN
    return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

constexpr int GK = 32;       // K chunk
constexpr int GKP = GK + 8;  // LDS row pitch (bf16 values): 80 bytes

template <bool TA, bool TB>
__global__ void __launch_bounds__(256, 4) k_gemm(int M, int N, int K, const float* __restrict__ A, int lda,
                                              const float* __restrict__ B, int ldb, float* __restrict__ Cm, int ldc,
                                              int beta, const float* __restrict__ bias, int act,
                                              float* __restrict__ Z) {
  __shared__ __attribute__((aligned(16))) unsigned short As[64][GKP];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[64][GKP];
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int nsplit = gridDim.z;
  const int kchunk = ((K + nsplit - 1) / nsplit + GK - 1) / GK * GK;
  const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += GK) {
#pragma unroll
    for (int q = 0; q < 64 * GK / 256; ++q) {
      const int e = tid + 256 * q;
      // thread -> element maps that read consecutive addresses
      const int mm = TA ? e % 64 : e / GK, ka = TA ? e / 64 : e % GK;
      const int gm = m0 + mm, gka = k0 + ka;
      float va = 0.f;
      if (gm < M && gka < ke) va = TA ? A[(int64_t)gka * lda + gm] : A[(int64_t)gm * lda + gka];
      As[mm][ka] = bf16_bits(va);
      const int nn = TB ? e / GK : e % 64, kb2 = TB ? e % GK : e / 64;
      const int gn = n0 + nn, gkb = k0 + kb2;
      float vb = 0.f;
      if (gn < N && gkb < ke) vb = TB ? B[(int64_t)gn * ldb + gkb] : B[(int64_t)gkb * ldb + gn];
      Bs[nn][kb2] = bf16_bits(vb);
    }
    __syncthreads();
    bf16x8_t av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
      av[a] = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const uint4*>(&As[wr + 16 * a + (lane & 15)][8 * (lane >> 4)]));
#pragma unroll
    for (int b = 0; b < 2; ++b)
      bv[b] = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const uint4*>(&Bs[wc + 16 * b + (lane & 15)][8 * (lane >> 4)]));
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
    __syncthreads();
  }
  float* Cz = Cm + (int64_t)blockIdx.z * M * ldc;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wr + 16 * a + acc_row<float>(lane, r);
        const int gn = n0 + wc + 16 * b + (lane & 15);
        if (gm < M && gn < N) {
          float v = acc[a][b][r];
          float* cp = Cz + (int64_t)gm * ldc + gn;
          if (beta) v += *cp;
          if (bias) v += bias[gn];
          if (act) {
            if (Z) Z[(int64_t)gm * ldc + gn] = v;
            v = gelu_f(v);
          }
          *cp = v;
        }
      }
}

// sum of split-K slices: C[e] = sum_z W[z][e] (+ C[e] if beta)
__global__ void k_sum_splits(int64_t n, int nsplit, const float* __restrict__ W, float* __restrict__ C, int beta) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  float s = beta ? C[e] : 0.f;
  for (int z = 0; z < nsplit; ++z) s += W[(int64_t)z * n + e];
  C[e] = s;
}

// neighbour mean over subdomain adjacency within each graph (rows g*nsub + i)
__global__ void k_nbr_mean(int ngraph, int nsub, int F, const int64_t* __restrict__ nptr,
                           const int32_t* __restrict__ nbrs, const float* __restrict__ in, float* __restrict__ out) {
  int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)ngraph * nsub * F) return;
  int f = (int)(idx % F);
  int64_t node = idx / F;
  int i = (int)(node % nsub);
  int64_t g = node / nsub;
  int64_t a = nptr[i], b = nptr[i + 1];
  float s = 0.f;
  for (int64_t q = a; q < b; ++q) s += in[(g * nsub + nbrs[q]) * F + f];
  out[idx] = b > a ? s / (float)(b - a) : 0.f;
}

// adjoint of the neighbour mean: out[j] (+)= sum_{i in N(j)} in[i] / |N(i)|
__global__ void k_nbr_mean_T(int ngraph, int nsub, int F, const int64_t* __restrict__ nptr,
                             const int32_t* __restrict__ nbrs, const float* __restrict__ in, float* __restrict__ out,
                             int accumulate) {
  int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)ngraph * nsub * F) return;
  int f = (int)(idx % F);
  int64_t node = idx / F;
  int j = (int)(node % nsub);
  int64_t g = node / nsub;
  float s = 0.f;
  for (int64_t q = nptr[j]; q < nptr[j + 1]; ++q) {
    int i = nbrs[q];
    float cnt = (float)(nptr[i + 1] - nptr[i]);
    s += in[(g * nsub + i) * F + f] / cnt;
  }
  out[idx] = accumulate ? out[idx] + s : s;
}

__global__ void k_gelu_back(int64_t n, const float* __restrict__ dh, const float* __restrict__ z,
                            float* __restrict__ dz) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < n) dz[e] = dh[e] * gelu_grad_f(z[e]);
}

// d = 2 (out - y) / n, per-block partial sums of (out - y)^2
__global__ void __launch_bounds__(256) k_mse(int64_t n, const float* __restrict__ out, const float* __restrict__ y,
                                             float* __restrict__ d, double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    float diff = out[e] - y[e];
    d[e] = 2.f * diff / (float)n;
    s += (double)diff * diff;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// column sums: out[f] = sum_r in[r][f]  (bias gradients), fixed order
__global__ void k_colsum(int rows, int F, const float* __restrict__ in, float* __restrict__ out) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  double s = 0;
  for (int r = 0; r < rows; ++r) s += in[(int64_t)r * F + f];
  out[f] = (float)s;
}

__global__ void k_adam(int64_t n, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  float gg = g[e];
  float mm = b1 * m[e] + (1.f - b1) * gg;
  float vv = b2 * v[e] + (1.f - b2) * gg * gg;
  m[e] = mm;
  v[e] = vv;
  w[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

__global__ void k_gather_rows(int nrows_out, int F, const int32_t* __restrict__ graphs, int nsub,
                              const float* __restrict__ src, float* __restrict__ dst) {
  int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nrows_out * F) return;
  int f = (int)(idx % F);
  int64_t r = idx / F;
  int64_t g = r / nsub, i = r % nsub;
  dst[idx] = src[((int64_t)graphs[g] * nsub + i) * F + f];
}

__global__ void k_scale_f(int64_t n, float* __restrict__ x, float s) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < n) x[e] *= s;
}

__global__ void k_nonfinite(int64_t n, const float* __restrict__ x, int32_t* __restrict__ flag) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < n && !isfinite(x[e])) *flag = 1;
}

}  // namespace

void launch_coarse_P(hipStream_t s, int64_t nrows, const int32_t* row_sub, const int32_t* dofs, const int32_t* edges,
                     const double* xyz, const double* box, float* P) {
  if (nrows > 0)
    hipLaunchKernelGGL(k_coarse_P, dim3(nblk(nrows, 128)), dim3(128), 0, s, nrows, row_sub, dofs, edges, xyz, box, P);
}

int64_t pool_scratch_floats(int nsub) { return (int64_t)PS * 32 * nsub * NIN; }

void launch_pool(hipStream_t s, int nsub, const int64_t* dof_ptr, const int32_t* dofs, const float* P,
                 const double* wts, const double2* v, int nrhs, const double* scale, float* X, float* part) {
  for (int j0 = 0; j0 < nrhs; j0 += 32) {
    int nj = nrhs - j0 < 32 ? nrhs - j0 : 32;
    if (wts)
      hipLaunchKernelGGL(k_pool_part<true>, dim3(nsub, PS), dim3(256), 0, s, nsub, dof_ptr, dofs, P, wts, v, nrhs, j0,
                         nj, part);
    else
      hipLaunchKernelGGL(k_pool_part<false>, dim3(nsub, PS), dim3(256), 0, s, nsub, dof_ptr, dofs, P, wts, v, nrhs,
                         j0, nj, part);
    hipLaunchKernelGGL(k_pool_sum, dim3(nblk((int64_t)nj * nsub * NIN, 256)), dim3(256), 0, s, nsub, j0, nj, scale,
                       part, X, (int64_t)NIN);
  }
}

template <typename C>
void launch_coarse_apply(hipStream_t s, int64_t nrows, const int32_t* lpos, const int64_t* dof_ptr,
                         const int64_t* vec_off, const float* P, const float* Cn, int nsub, int nrhs,
                         const double* scale, float alpha, C* xloc) {
  if (nrows <= 0 || nsub <= 0) return;
  for (int j0 = 0; j0 < nrhs; j0 += 32) {
    const int nj = nrhs - j0 < 32 ? nrhs - j0 : 32;
    hipLaunchKernelGGL(k_coarse_apply<C>, dim3(nsub, 8), dim3(256), 0, s, lpos, dof_ptr, vec_off, P, Cn, nsub, nrhs,
                       j0, nj, scale, alpha, xloc);
  }
}
template void launch_coarse_apply<float2>(hipStream_t, int64_t, const int32_t*, const int64_t*, const int64_t*,
                                          const float*, const float*, int, int, const double*, float, float2*);
template void launch_coarse_apply<double2>(hipStream_t, int64_t, const int32_t*, const int64_t*, const int64_t*,
                                           const float*, const float*, int, int, const double*, float, double2*);

void launch_gapply(hipStream_t s, int nsub, int nrhs, const double* G, const float* in, float* out) {
  hipLaunchKernelGGL(k_gapply, dim3(nsub, nrhs), dim3(NCO), 0, s, nsub, nrhs, G, in, out);
}
void launch_pdp(hipStream_t s, int nsub, const int64_t* dof_ptr, const float* P, const double* D, double* out) {
  hipLaunchKernelGGL(k_pdp, dim3(nsub, NCO), dim3(NCO), 0, s, dof_ptr, P, D, out);
}

void launch_gemm(hipStream_t s, bool ta, bool tb, int M, int N, int K, const float* A, int lda, const float* B,
                 int ldb, float* C, int ldc, int beta, const float* bias, int act, float* Z, int rnd, int nsplit,
                 float* work) {
  if (M <= 0 || N <= 0) return;
  dim3 grid(nblk(N, 64), nblk(M, 64), 1);
  float* out = C;
  int b = beta;
  if (nsplit > 1) {
    grid.z = nsplit;
    out = work;
    b = 0;
  }
  (void)rnd;  // operands are always rounded to bf16 (the network's arithmetic)
#define MXG(TA_, TB_) \
  hipLaunchKernelGGL((k_gemm<TA_, TB_>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, out, ldc, b, \
                     nsplit > 1 ? nullptr : bias, nsplit > 1 ? 0 : act, Z)
  if (!ta && !tb) MXG(false, false);
  else if (!ta && tb) MXG(false, true);
  else if (ta && !tb) MXG(true, false);
  else MXG(true, true);
#undef MXG
  if (nsplit > 1) {
    int64_t n = (int64_t)M * ldc;
    hipLaunchKernelGGL(k_sum_splits, dim3(nblk(n, 256)), dim3(256), 0, s, n, nsplit, work, C, beta);
  }
}

void launch_nbr_mean(hipStream_t s, int ngraph, int nsub, int F, const int64_t* nptr, const int32_t* nbrs,
                     const float* in, float* out) {
  int64_t n = (int64_t)ngraph * nsub * F;
  if (n > 0) hipLaunchKernelGGL(k_nbr_mean, dim3(nblk(n, 256)), dim3(256), 0, s, ngraph, nsub, F, nptr, nbrs, in, out);
}
void launch_nbr_mean_T(hipStream_t s, int ngraph, int nsub, int F, const int64_t* nptr, const int32_t* nbrs,
                       const float* in, float* out, int accumulate) {
  int64_t n = (int64_t)ngraph * nsub * F;
  if (n > 0)
    hipLaunchKernelGGL(k_nbr_mean_T, dim3(nblk(n, 256)), dim3(256), 0, s, ngraph, nsub, F, nptr, nbrs, in, out,
                       accumulate);
}
void launch_gelu_back(hipStream_t s, int64_t n, const float* dh, const float* z, float* dz) {
  if (n > 0) hipLaunchKernelGGL(k_gelu_back, dim3(nblk(n, 256)), dim3(256), 0, s, n, dh, z, dz);
}
int mse_blocks() { return 256; }
void launch_mse(hipStream_t s, int64_t n, const float* out, const float* y, float* d, double* part) {
  hipLaunchKernelGGL(k_mse, dim3(256), dim3(256), 0, s, n, out, y, d, part);
}
void launch_colsum(hipStream_t s, int rows, int F, const float* in, float* out) {
  hipLaunchKernelGGL(k_colsum, dim3(nblk(F, 128)), dim3(128), 0, s, rows, F, in, out);
}
void launch_adam(hipStream_t s, int64_t n, float* w, const float* g, float* m, float* v, float lr, float b1, float b2,
                 float eps, int t) {
  float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  if (n > 0) hipLaunchKernelGGL(k_adam, dim3(nblk(n, 256)), dim3(256), 0, s, n, w, g, m, v, lr, b1, b2, eps, c1, c2);
}
void launch_gather_rows(hipStream_t s, int nrows_out, int F, const int32_t* graphs, int nsub, const float* src,
                        float* dst) {
  int64_t n = (int64_t)nrows_out * F;
  if (n > 0) hipLaunchKernelGGL(k_gather_rows, dim3(nblk(n, 256)), dim3(256), 0, s, nrows_out, F, graphs, nsub, src, dst);
}
void launch_scale_f(hipStream_t s, int64_t n, float* x, float f) {
  if (n > 0) hipLaunchKernelGGL(k_scale_f, dim3(nblk(n, 256)), dim3(256), 0, s, n, x, f);
}
void launch_nonfinite(hipStream_t s, int64_t n, const float* x, int32_t* flag) {
  if (n > 0) hipLaunchKernelGGL(k_nonfinite, dim3(nblk(n, 256)), dim3(256), 0, s, n, x, flag);
}

}  // namespace mx
