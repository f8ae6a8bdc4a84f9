// Pseudo-block flexible GMRES building blocks (complex128): classical
// Gram-Schmidt dot products with deterministic two-stage reductions, vector
// updates, per-right-hand-side Givens rotations and least-squares updates,
// plus the dipole right-hand sides and receiver functionals.
//
// Block vectors are DOF-major [n][nrhs]; the Krylov bases are arrays of such
// blocks with stride vstride elements.
#include "mx_device.h"
#include "mx_kernels.h"

namespace mx {

namespace {

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// part[b][i][j] = sum over this block's rows of conj(V_{i0+i}[r][j]) w[r][j]
template <int NV>
__global__ void __launch_bounds__(256) k_dot(int64_t nrows, int nrhs, const double2* __restrict__ V, int64_t vstride,
                                             int i0, const double2* __restrict__ w, double2* __restrict__ part) {
  const int rpi = blockDim.x / nrhs;
  const int t = threadIdx.x;
  const int j = t % nrhs, rl = t / nrhs;
  const int64_t chunk = (nrows + gridDim.x - 1) / gridDim.x;
  const int64_t rb = blockIdx.x * chunk, re = min(nrows, rb + chunk);
  double ar[NV], ai[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) { ar[i] = 0; ai[i] = 0; }
  if (rl < rpi) {
    for (int64_t r = rb + rl; r < re; r += rpi) {
      const int64_t o = r * nrhs + j;
      double2 x = w[o];
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        double2 v = V[(int64_t)(i0 + i) * vstride + o];
        ar[i] += v.x * x.x + v.y * x.y;
        ai[i] += v.x * x.y - v.y * x.x;
      }
    }
  }
  __shared__ double2 red[256];
  for (int i = 0; i < NV; ++i) {
    red[t] = make_double2(ar[i], ai[i]);
    __syncthreads();
    if (rl == 0 && t < nrhs) {
      double sr = 0, si = 0;
      for (int q = 0; q < rpi; ++q) {
        sr += red[q * nrhs + j].x;
        si += red[q * nrhs + j].y;
      }
      part[((int64_t)blockIdx.x * NV + i) * nrhs + j] = make_double2(sr, si);
    }
    __syncthreads();
  }
}

// out[(o0 + i) * nrhs + j] = sum_b part[b][i][j] (fixed order)
__global__ void k_dot_final(int nb, int nv, int nrhs, const double2* __restrict__ part, double2* __restrict__ out,
                            int o0) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nv * nrhs) return;
  int i = idx / nrhs, j = idx % nrhs;
  double sr = 0, si = 0;
  for (int b = 0; b < nb; ++b) {
    double2 p = part[((int64_t)b * nv + i) * nrhs + j];
    sr += p.x;
    si += p.y;
  }
  out[(int64_t)(o0 + i) * nrhs + j] = make_double2(sr, si);
}

// w[r][j] -= sum_{i < nv} V_i[r][j] h[i][j]
__global__ void k_update(int64_t nrows, int nrhs, const double2* __restrict__ V, int64_t vstride, int nv,
                         const double2* __restrict__ h, double2* __restrict__ w) {
  int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= nrows * nrhs) return;
  int j = (int)(idx % nrhs);
  double2 acc = w[idx];
  for (int i = 0; i < nv; ++i) {
    double2 v = V[(int64_t)i * vstride + idx];
    double2 hh = h[i * nrhs + j];
    acc.x -= v.x * hh.x - v.y * hh.y;
    acc.y -= v.x * hh.y + v.y * hh.x;
  }
  w[idx] = acc;
}

// Fused Gram-Schmidt passes. Both take w <- w - sum_{i < NV} V_i h[i] (the
// same arithmetic and order as k_update) and then, on the updated rows,
// MODE 0: part[b][i][j] = sum over this block's rows of conj(V_i[r][j]) w[r][j]
//         (the next pass's coefficients, same row split and order as k_dot),
// MODE 1: npart[b][j] = sum over this block's rows of |w[r][j]|^2 (as k_norm2).
// The V_i values of a row stay in registers between the update and the dot,
// so each basis vector is read once per pass instead of twice.
// MODE 2: no update; the MODE 0 dots of w itself, all NV in one sweep (w read
// once instead of once per 8 basis vectors as in k_dot).
template <int NV, int MODE>
__global__ void __launch_bounds__(256) k_cgs_pass(int64_t nrows, int nrhs, const double2* __restrict__ V,
                                                  int64_t vstride, const double2* __restrict__ h,
                                                  double2* __restrict__ w, double2* __restrict__ part,
                                                  double* __restrict__ npart) {
  const int rpi = blockDim.x / nrhs;
  const int t = threadIdx.x;
  const int j = t % nrhs, rl = t / nrhs;
  const int64_t chunk = (nrows + gridDim.x - 1) / gridDim.x;
  const int64_t rb = blockIdx.x * chunk, re = min(nrows, rb + chunk);
  __shared__ double2 hs[NV][32];
  if (MODE != 2)
    for (int e = t; e < NV * nrhs; e += blockDim.x) hs[e / nrhs][e % nrhs] = h[e];
  __syncthreads();
  double ar[MODE != 1 ? NV : 1], ai[MODE != 1 ? NV : 1];
  double a2 = 0;
#pragma unroll
  for (int i = 0; i < (MODE != 1 ? NV : 1); ++i) { ar[i] = 0; ai[i] = 0; }
  if (rl < rpi) {
#pragma unroll 1
    for (int64_t r = rb + rl; r < re; r += rpi) {
      const int64_t o = r * nrhs + j;
      double2 v[NV];
#pragma unroll
      for (int i = 0; i < NV; ++i) v[i] = V[(int64_t)i * vstride + o];
      double2 acc = w[o];
      if (MODE != 2) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
          const double2 hh = hs[i][j];
          acc.x -= v[i].x * hh.x - v[i].y * hh.y;
          acc.y -= v[i].x * hh.y + v[i].y * hh.x;
        }
        w[o] = acc;
      }
      if (MODE != 1) {
#pragma unroll
        for (int i = 0; i < (MODE != 1 ? NV : 1); ++i) {
          ar[i] += v[i].x * acc.x + v[i].y * acc.y;
          ai[i] += v[i].x * acc.y - v[i].y * acc.x;
        }
      } else {
        a2 += acc.x * acc.x + acc.y * acc.y;
      }
    }
  }
  if (MODE != 1) {
    __shared__ double2 red[256];
    for (int i = 0; i < NV; ++i) {
      red[t] = make_double2(ar[i], ai[i]);
      __syncthreads();
      if (rl == 0 && t < nrhs) {
        double sr = 0, si = 0;
        for (int q = 0; q < rpi; ++q) {
          sr += red[q * nrhs + j].x;
          si += red[q * nrhs + j].y;
        }
        part[((int64_t)blockIdx.x * NV + i) * nrhs + j] = make_double2(sr, si);
      }
      __syncthreads();
    }
  } else {
    __shared__ double redn[256];
    redn[t] = a2;
    __syncthreads();
    if (rl == 0 && t < nrhs) {
      double sum = 0;
      for (int q = 0; q < rpi; ++q) sum += redn[q * nrhs + j];
      npart[(int64_t)blockIdx.x * nrhs + j] = sum;
    }
  }
}

// part[b][j] = sum over this block's rows of |w[r][j]|^2
__global__ void __launch_bounds__(256) k_norm2(int64_t nrows, int nrhs, const double2* __restrict__ w,
                                               double* __restrict__ part) {
  const int rpi = blockDim.x / nrhs;
  const int t = threadIdx.x;
  const int j = t % nrhs, rl = t / nrhs;
  const int64_t chunk = (nrows + gridDim.x - 1) / gridDim.x;
  const int64_t rb = blockIdx.x * chunk, re = min(nrows, rb + chunk);
  double a = 0;
  if (rl < rpi)
    for (int64_t r = rb + rl; r < re; r += rpi) {
      double2 x = w[r * nrhs + j];
      a += x.x * x.x + x.y * x.y;
    }
  __shared__ double red[256];
  red[t] = a;
  __syncthreads();
  if (rl == 0 && t < nrhs) {
    double s = 0;
    for (int q = 0; q < rpi; ++q) s += red[q * nrhs + j];
    part[(int64_t)blockIdx.x * nrhs + j] = s;
  }
}

__global__ void k_norm_final(int nb, int nrhs, const double* __restrict__ part, double* __restrict__ out) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nrhs) return;
  double s = 0;
  for (int b = 0; b < nb; ++b) s += part[(int64_t)b * nrhs + j];
  out[j] = sqrt(s);
}

// dst[r][j] = src[r][j] * (nrm[j] > 0 ? 1/nrm[j] : 0)
__global__ void k_scale(int64_t nrows, int nrhs, const double2* __restrict__ src, const double* __restrict__ nrm,
                        double2* __restrict__ dst) {
  int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= nrows * nrhs) return;
  double n = nrm[idx % nrhs];
  double s = n > 0 ? 1.0 / n : 0.0;
  double2 x = src[idx];
  dst[idx] = make_double2(x.x * s, x.y * s);
}

// r = b - r
__global__ void k_bminus(int64_t n, const double2* __restrict__ b, double2* __restrict__ r) {
  int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= n) return;
  double2 x = r[idx], y = b[idx];
  r[idx] = make_double2(y.x - x.x, y.y - x.y);
}

__device__ inline void givens(double2 a, double2 b, double& c, double2& s) {
  double aa = hypot(a.x, a.y), bb = hypot(b.x, b.y);
  if (bb == 0) { c = 1; s = make_double2(0, 0); return; }
  if (aa == 0) { c = 0; s = make_double2(b.x / bb, -b.y / bb); return; }
  double den = hypot(aa, bb);
  c = aa / den;
  // s = (a/|a|) conj(b) / den
  double2 ua = make_double2(a.x / aa, a.y / aa);
  s = make_double2((ua.x * b.x + ua.y * b.y) / den, (ua.y * b.x - ua.x * b.y) / den);
}

// Column k of the Hessenberg matrix for every right-hand side: store h1 + h2
// and ||w||, apply the previous rotations, form the new one, update g and the
// residual estimate |g_{k+1}| / ||b||.
__global__ void k_givens(int k, int m, int nrhs, const double2* __restrict__ h1, const double2* __restrict__ h2,
                         const double* __restrict__ hn, double2* __restrict__ H, double* __restrict__ cs,
                         double2* __restrict__ sn, double2* __restrict__ g, const double* __restrict__ bnorm,
                         double rtol, int32_t* __restrict__ conv, int32_t* __restrict__ kdone,
                         double* __restrict__ res) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nrhs) return;
#define HH(i, kk) H[((int64_t)(i) * m + (kk)) * nrhs + j]
  for (int i = 0; i <= k; ++i) {
    double2 a = h1[i * nrhs + j], b = h2[i * nrhs + j];
    HH(i, k) = make_double2(a.x + b.x, a.y + b.y);
  }
  HH(k + 1, k) = make_double2(hn[j], 0.0);
  for (int i = 0; i < k; ++i) {
    double c = cs[i * nrhs + j];
    double2 s = sn[i * nrhs + j];
    double2 x = HH(i, k), y = HH(i + 1, k);
    double2 t = make_double2(c * x.x + s.x * y.x - s.y * y.y, c * x.y + s.x * y.y + s.y * y.x);
    // -conj(s) x + c y
    double2 u = make_double2(-(s.x * x.x + s.y * x.y) + c * y.x, -(s.x * x.y - s.y * x.x) + c * y.y);
    HH(i, k) = t;
    HH(i + 1, k) = u;
  }
  double c;
  double2 s;
  double2 a = HH(k, k), b = HH(k + 1, k);
  givens(a, b, c, s);
  HH(k, k) = make_double2(c * a.x + s.x * b.x - s.y * b.y, c * a.y + s.x * b.y + s.y * b.x);
  HH(k + 1, k) = make_double2(0, 0);
  cs[k * nrhs + j] = c;
  sn[k * nrhs + j] = s;
  double2 gk = g[k * nrhs + j];
  g[(k + 1) * nrhs + j] = make_double2(-(s.x * gk.x + s.y * gk.y), -(s.x * gk.y - s.y * gk.x));
  g[k * nrhs + j] = make_double2(c * gk.x, c * gk.y);
  double2 gn = g[(k + 1) * nrhs + j];
  double rr = bnorm[j] > 0 ? hypot(gn.x, gn.y) / bnorm[j] : 0.0;
  res[j] = rr;
  // a zero right-hand side has the zero solution: no step contributes
  if (!conv[j] && rr <= rtol) { conv[j] = 1; kdone[j] = bnorm[j] > 0 ? k + 1 : 0; }
#undef HH
}

// y = H^{-1} g on the first kd columns (kd = kdone if converged in this cycle,
// else ksteps)
__global__ void k_lsq(int ksteps, int m, int nrhs, const double2* __restrict__ H, const double2* __restrict__ g,
                      const int32_t* __restrict__ conv, int32_t* __restrict__ kdone, double2* __restrict__ y) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nrhs) return;
  int kd = conv[j] ? kdone[j] : ksteps;
  kdone[j] = kd;
  for (int i = kd - 1; i >= 0; --i) {
    double2 acc = g[i * nrhs + j];
    for (int l = i + 1; l < kd; ++l) {
      double2 h = H[((int64_t)i * m + l) * nrhs + j], yy = y[l * nrhs + j];
      acc.x -= h.x * yy.x - h.y * yy.y;
      acc.y -= h.x * yy.y + h.y * yy.x;
    }
    double2 d = H[((int64_t)i * m + i) * nrhs + j];
    // an exactly singular rotated Hessenberg (breakdown) contributes nothing
    y[i * nrhs + j] = (d.x != 0.0 || d.y != 0.0) ? cdiv(acc, d) : make_double2(0.0, 0.0);
  }
}

// x[r][j] += sum_{i < kd[j]} Z_i[r][j] y[i][j]
__global__ void k_xupdate(int64_t nrows, int nrhs, const double2* __restrict__ Z, int64_t vstride,
                          const double2* __restrict__ y, const int32_t* __restrict__ kd, double2* __restrict__ x) {
  int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= nrows * nrhs) return;
  int j = (int)(idx % nrhs);
  int n = kd[j];
  double2 acc = x[idx];
  for (int i = 0; i < n; ++i) {
    double2 z = Z[(int64_t)i * vstride + idx], yy = y[i * nrhs + j];
    acc.x += z.x * yy.x - z.y * yy.y;
    acc.y += z.x * yy.y + z.y * yy.x;
  }
  x[idx] = acc;
}

// B[edge[k]][col[k]] = scale * val[k]  (entries are distinct)
__global__ void k_scatter_rhs(int64_t n, const int32_t* __restrict__ edge, const int32_t* __restrict__ col,
                              const double2* __restrict__ val, double2 scale, int nrhs, double2* __restrict__ B) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  double2 v = val[k];
  B[(int64_t)edge[k] * nrhs + col[k]] = make_double2(scale.x * v.x - scale.y * v.y, scale.x * v.y + scale.y * v.x);
}

// S[i][j] = sum_k val_i[k] U[edge_i[k]][j]
__global__ void k_receivers(int nrx, int nrhs, const int64_t* __restrict__ ptr, const int32_t* __restrict__ edge,
                            const double2* __restrict__ val, const double2* __restrict__ U, double2* __restrict__ S) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nrx * nrhs) return;
  int i = idx / nrhs, j = idx % nrhs;
  double sr = 0, si = 0;
  for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
    double2 v = val[k], u = U[(int64_t)edge[k] * nrhs + j];
    sr += v.x * u.x - v.y * u.y;
    si += v.x * u.y + v.y * u.x;
  }
  S[idx] = make_double2(sr, si);
}

}  // namespace

int dot_blocks(int64_t nrows) {
  int64_t b = (nrows + 2047) / 2048;
  return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

void launch_dot(hipStream_t s, int64_t nrows, int nrhs, const double2* V, int64_t vstride, int nvec,
                const double2* w, double2* part, double2* out) {
  const int nb = dot_blocks(nrows);
  const int rpi = nrhs <= 256 ? 256 / nrhs : 1;
  const int threads = rpi * nrhs;
  for (int i0 = 0; i0 < nvec; i0 += 8) {
    const int nv = nvec - i0 < 8 ? nvec - i0 : 8;
    switch (nv) {
#define MXCASE(K)                                                                                        \
  case K:                                                                                                \
    hipLaunchKernelGGL(k_dot<K>, dim3(nb), dim3(threads), 0, s, nrows, nrhs, V, vstride, i0, w, part); \
    break;
      MXCASE(1) MXCASE(2) MXCASE(3) MXCASE(4) MXCASE(5) MXCASE(6) MXCASE(7) MXCASE(8)
#undef MXCASE
    }
    hipLaunchKernelGGL(k_dot_final, dim3(nblk(nv * nrhs, 256)), dim3(256), 0, s, nb, nv, nrhs, part, out, i0);
  }
}

int cgs_fused_max() { return 32; }

int launch_cgs_pass(hipStream_t s, int64_t nrows, int nrhs, const double2* V, int64_t vstride, int nv,
                    const double2* h, double2* w, double2* part, double* npart, double2* hout, double* nout) {
  if (nv < 1 || nv > 32 || nrhs > 32 || nrhs < 1) return -1;
  const int nb = dot_blocks(nrows);
  const int rpi = 256 / nrhs;
  const int threads = rpi * nrhs;
  const bool dot = hout != nullptr;
  const bool upd = h != nullptr;
  switch (nv) {
#define MXC(K)                                                                                                    \
  case K:                                                                                                         \
    if (dot && !upd)                                                                                              \
      hipLaunchKernelGGL((k_cgs_pass<K, 2>), dim3(nb), dim3(threads), 0, s, nrows, nrhs, V, vstride, h, w, part, \
                         npart);                                                                                  \
    else if (dot)                                                                                                 \
      hipLaunchKernelGGL((k_cgs_pass<K, 0>), dim3(nb), dim3(threads), 0, s, nrows, nrhs, V, vstride, h, w, part, \
                         npart);                                                                                  \
    else                                                                                                          \
      hipLaunchKernelGGL((k_cgs_pass<K, 1>), dim3(nb), dim3(threads), 0, s, nrows, nrhs, V, vstride, h, w, part, \
                         npart);                                                                                  \
    break;
    MXC(1) MXC(2) MXC(3) MXC(4) MXC(5) MXC(6) MXC(7) MXC(8) MXC(9) MXC(10) MXC(11) MXC(12) MXC(13) MXC(14)
    MXC(15) MXC(16) MXC(17) MXC(18) MXC(19) MXC(20) MXC(21) MXC(22) MXC(23) MXC(24) MXC(25) MXC(26) MXC(27)
    MXC(28) MXC(29) MXC(30) MXC(31) MXC(32)
#undef MXC
  }
  if (dot)
    hipLaunchKernelGGL(k_dot_final, dim3(nblk(nv * nrhs, 256)), dim3(256), 0, s, nb, nv, nrhs, part, hout, 0);
  else
    hipLaunchKernelGGL(k_norm_final, dim3(nblk(nrhs, 256)), dim3(256), 0, s, nb, nrhs, npart, nout);
  return 0;
}

void launch_update(hipStream_t s, int64_t nrows, int nrhs, const double2* V, int64_t vstride, int nv,
                   const double2* h, double2* w) {
  int64_t n = nrows * nrhs;
  if (n > 0 && nv > 0) hipLaunchKernelGGL(k_update, dim3(nblk(n, 256)), dim3(256), 0, s, nrows, nrhs, V, vstride, nv, h, w);
}

void launch_norm(hipStream_t s, int64_t nrows, int nrhs, const double2* w, double* part, double* out) {
  const int nb = dot_blocks(nrows);
  const int rpi = nrhs <= 256 ? 256 / nrhs : 1;
  hipLaunchKernelGGL(k_norm2, dim3(nb), dim3(rpi * nrhs), 0, s, nrows, nrhs, w, part);
  hipLaunchKernelGGL(k_norm_final, dim3(nblk(nrhs, 256)), dim3(256), 0, s, nb, nrhs, part, out);
}

void launch_scale(hipStream_t s, int64_t nrows, int nrhs, const double2* src, const double* nrm, double2* dst) {
  int64_t n = nrows * nrhs;
  if (n > 0) hipLaunchKernelGGL(k_scale, dim3(nblk(n, 256)), dim3(256), 0, s, nrows, nrhs, src, nrm, dst);
}

void launch_bminus(hipStream_t s, int64_t n, const double2* b, double2* r) {
  if (n > 0) hipLaunchKernelGGL(k_bminus, dim3(nblk(n, 256)), dim3(256), 0, s, n, b, r);
}

void launch_givens(hipStream_t s, int k, int m, int nrhs, const double2* h1, const double2* h2, const double* hn,
                   double2* H, double* cs, double2* sn, double2* g, const double* bnorm, double rtol, int32_t* conv,
                   int32_t* kdone, double* res) {
  hipLaunchKernelGGL(k_givens, dim3(nblk(nrhs, 64)), dim3(64), 0, s, k, m, nrhs, h1, h2, hn, H, cs, sn, g, bnorm,
                     rtol, conv, kdone, res);
}

void launch_lsq(hipStream_t s, int ksteps, int m, int nrhs, const double2* H, const double2* g, const int32_t* conv,
                int32_t* kdone, double2* y) {
  hipLaunchKernelGGL(k_lsq, dim3(nblk(nrhs, 64)), dim3(64), 0, s, ksteps, m, nrhs, H, g, conv, kdone, y);
}

void launch_xupdate(hipStream_t s, int64_t nrows, int nrhs, const double2* Z, int64_t vstride, const double2* y,
                    const int32_t* kd, double2* x) {
  int64_t n = nrows * nrhs;
  if (n > 0) hipLaunchKernelGGL(k_xupdate, dim3(nblk(n, 256)), dim3(256), 0, s, nrows, nrhs, Z, vstride, y, kd, x);
}

void launch_scatter_rhs(hipStream_t s, int64_t n, const int32_t* edge, const int32_t* col, const double2* val,
                        double2 scale, int nrhs, double2* B) {
  if (n > 0) hipLaunchKernelGGL(k_scatter_rhs, dim3(nblk(n, 256)), dim3(256), 0, s, n, edge, col, val, scale, nrhs, B);
}

void launch_receivers(hipStream_t s, int nrx, int nrhs, const int64_t* ptr, const int32_t* edge, const double2* val,
                      const double2* U, double2* S) {
  int n = nrx * nrhs;
  if (n > 0) hipLaunchKernelGGL(k_receivers, dim3(nblk(n, 256)), dim3(256), 0, s, nrx, nrhs, ptr, edge, val, U, S);
}

}  // namespace mx
