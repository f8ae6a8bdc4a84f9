// Operator kernels: element and face blocks of the weak form (2), their
// deterministic gather into the global CSR matrix and into the dense ORAS
// subdomain matrices, the complex block SpMM, and the partition-of-unity
// restriction / prolongation.
#include "mx_device.h"
#include "mx_kernels.h"

namespace mx {

namespace {

__constant__ int cLE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
__constant__ int cLF[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};
__constant__ int cFE2[3][2] = {{0, 1}, {0, 2}, {1, 2}};

__device__ inline void sub3(const double* a, const double* b, double* o) {
  o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
__device__ inline void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ inline double dot3(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Barycentric gradients from face normals: grad l_k is parallel to the normal
// N_k of the face opposite vertex k and grad l_k . (x_k - x_j) = 1 for any
// vertex j of that face.  Returns the volume |T|.
__device__ double tet_geometry(const double* xyz, const int32_t* v, double g[4][3]) {
  double X[4][3];
  for (int k = 0; k < 4; ++k)
    for (int c = 0; c < 3; ++c) X[k][c] = xyz[3 * (size_t)v[k] + c];
  for (int k = 0; k < 4; ++k) {
    int j0 = (k + 1) & 3, j1 = (k + 2) & 3, j2 = (k + 3) & 3;
    double u[3], w[3], n[3], d[3];
    sub3(X[j1], X[j0], u);
    sub3(X[j2], X[j0], w);
    cross3(u, w, n);
    sub3(X[k], X[j0], d);
    double den = dot3(n, d);
    for (int c = 0; c < 3; ++c) g[k][c] = n[c] / den;
  }
  double a[3], b[3], c[3], n[3];
  sub3(X[1], X[0], a);
  sub3(X[2], X[0], b);
  sub3(X[3], X[0], c);
  cross3(b, c, n);
  return fabs(dot3(a, n)) / 6.0;
}

// int_T l_n l_i l_j / |T| = (1 + d_ni + d_nj + d_ij + 2 d_ni d_ij) / 120
__device__ inline double lll(int n, int i, int j) {
  int dni = n == i, dnj = n == j, dij = i == j;
  return (1 + dni + dnj + dij + 2 * dni * dij) / 120.0;
}

__device__ inline double2 csqrt_principal(double2 z) {
  double r = hypot(z.x, z.y);
  double re = sqrt(0.5 * (r + z.x));
  double im = sqrt(fmax(0.5 * (r - z.x), 0.0));
  if (z.y < 0) im = -im;
  return make_double2(re, im);
}

// Element block K_T - k0^2 (eps M)_T (6x6, mirrored upper triangle).
__global__ void k_element(int32_t nt, const int32_t* __restrict__ ts, const double* __restrict__ xyz,
                          const double2* __restrict__ eps, int eps_kind, double k0sq,
                          double2* __restrict__ out) {
  int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  int32_t v[4];
  for (int k = 0; k < 4; ++k) v[k] = ts[4 * (size_t)t + k];
  double g[4][3];
  double vol = tet_geometry(xyz, v, g);
  double G[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) G[i][j] = dot3(g[i], g[j]);
  // W_ij = int_T eps l_i l_j
  double2 W[4][4];
  if (eps_kind == 0) {
    double2 e = eps[t];
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        double f = vol * (1 + (i == j)) / 20.0;
        W[i][j] = make_double2(e.x * f, e.y * f);
      }
  } else {
    double2 ev[4];
    for (int k = 0; k < 4; ++k) ev[k] = eps[v[k]];
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        double re = 0, im = 0;
        for (int n = 0; n < 4; ++n) {
          double f = lll(n, i, j);
          re += ev[n].x * f;
          im += ev[n].y * f;
        }
        W[i][j] = make_double2(vol * re, vol * im);
      }
  }
  double2* o = out + 36 * (size_t)t;
  for (int p = 0; p < 6; ++p) {
    int a = cLE[p][0], b = cLE[p][1];
    for (int q = p; q < 6; ++q) {
      int c = cLE[q][0], d = cLE[q][1];
      double K = 4.0 * vol * (G[a][c] * G[b][d] - G[a][d] * G[b][c]);
      double mre = W[a][c].x * G[b][d] - W[a][d].x * G[b][c] - W[b][c].x * G[a][d] + W[b][d].x * G[a][c];
      double mim = W[a][c].y * G[b][d] - W[a][d].y * G[b][c] - W[b][c].y * G[a][d] + W[b][d].y * G[a][c];
      double2 val = make_double2(K - k0sq * mre, -k0sq * mim);
      o[6 * p + q] = val;
      o[6 * q + p] = val;
    }
  }
}

// Face block j k B_F for (tet, local face) entries; k = kconst when
// per_tet_k == 0, else k0 sqrt(eps of the tetrahedron). A non-null kface
// gives k per face instead (port faces beta_p, metallic faces 0), taking
// precedence over kconst.
__global__ void k_face(int32_t n, const int32_t* __restrict__ ftet, const int32_t* __restrict__ flf,
                       const int32_t* __restrict__ ts, const double* __restrict__ xyz,
                       const double2* __restrict__ eps, int eps_kind, int per_tet_k, double k0,
                       double2 kconst, const double2* __restrict__ kface, double2* __restrict__ out) {
  int32_t f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n) return;
  int32_t t = ftet[f], lf = flf[f];
  int32_t v[4];
  for (int k = 0; k < 4; ++k) v[k] = ts[4 * (size_t)t + k];
  double g[4][3];
  tet_geometry(xyz, v, g);
  int fv[3] = {cLF[lf][0], cLF[lf][1], cLF[lf][2]};
  double P[3][3];
  for (int k = 0; k < 3; ++k)
    for (int c = 0; c < 3; ++c) P[k][c] = xyz[3 * (size_t)v[fv[k]] + c];
  double u[3], w[3], nrm[3];
  sub3(P[1], P[0], u);
  sub3(P[2], P[0], w);
  cross3(u, w, nrm);
  double nn = sqrt(dot3(nrm, nrm));
  double area = 0.5 * nn;
  for (int c = 0; c < 3; ++c) nrm[c] /= nn;
  double gs[3][3];
  for (int k = 0; k < 3; ++k) {
    double s = dot3(g[fv[k]], nrm);
    for (int c = 0; c < 3; ++c) gs[k][c] = g[fv[k]][c] - s * nrm[c];
  }
  double G[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) G[i][j] = dot3(gs[i], gs[j]);
  double2 kk = kface ? kface[f] : kconst;
  if (per_tet_k) {
    double2 e;
    if (eps_kind == 0) {
      e = eps[t];
    } else {
      double re = 0, im = 0;
      for (int k = 0; k < 4; ++k) { re += eps[v[k]].x; im += eps[v[k]].y; }
      e = make_double2(re / 4.0, im / 4.0);
    }
    double2 sq = csqrt_principal(e);
    kk = make_double2(k0 * sq.x, k0 * sq.y);
  }
  // j k = (-k.y, k.x)
  double2 jk = make_double2(-kk.y, kk.x);
  double2* o = out + 9 * (size_t)f;
  for (int p = 0; p < 3; ++p) {
    int a = cFE2[p][0], b = cFE2[p][1];
    for (int q = p; q < 3; ++q) {
      int c = cFE2[q][0], d = cFE2[q][1];
      double m = (1 + (a == c)) * G[b][d] - (1 + (a == d)) * G[b][c] - (1 + (b == c)) * G[a][d] +
                 (1 + (b == d)) * G[a][c];
      double B = area / 12.0 * m;
      double2 val = make_double2(jk.x * B, jk.y * B);
      o[3 * p + q] = val;
      o[3 * q + p] = val;
    }
  }
}

// Metallic edges eliminated symmetrically from the CSR operator: entries in a
// metallic row or column become 0, the diagonal of a metallic row 1.
__global__ void k_pec_csr(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                          const int32_t* __restrict__ pec, double2* __restrict__ val) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  const bool pr = pec[r] != 0;
  for (int64_t k = rp[r]; k < rp[r + 1]; ++k)
    if (pr || pec[col[k]] != 0) val[k] = make_double2(col[k] == r ? 1.0 : 0.0, 0.0);
}

// The same elimination in the dense subdomain matrices: for every metallic
// local index q of subdomain s, row q and column q are cleared and A[q][q] = 1.
template <typename C>
__global__ void k_pec_local(int32_t nsub, const int32_t* __restrict__ Npad, const int64_t* __restrict__ mat_off,
                            const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx, C* __restrict__ A) {
  const int s = blockIdx.x;
  if (s >= nsub) return;
  const int64_t N = Npad[s];
  C* M = A + mat_off[s];
  for (int64_t k = ptr[s]; k < ptr[s + 1]; ++k) {
    const int64_t q = idx[k];
    for (int64_t j = threadIdx.x; j < N; j += blockDim.x) {
      C v;
      v.x = j == q ? 1 : 0;
      v.y = 0;
      M[q * N + j] = v;
      M[j * N + q] = v;
    }
  }
}

// B[rows[k]][:] = 0
__global__ void k_zero_rows(int64_t n, const int32_t* __restrict__ rows, int nrhs, double2* __restrict__ B) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  B[(int64_t)rows[i / nrhs] * nrhs + i % nrhs] = make_double2(0.0, 0.0);
}

// out[k] = sum of pool[src[j]] for j in [ptr[k], ptr[k+1]) (fixed order)
__global__ void k_gather_csr(int64_t n, const int64_t* __restrict__ ptr, const int32_t* __restrict__ src,
                             const double2* __restrict__ pool, double2* __restrict__ out) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  double re = 0, im = 0;
  for (int64_t j = ptr[k]; j < ptr[k + 1]; ++j) {
    double2 v = pool[src[j]];
    re += v.x;
    im += v.y;
  }
  out[k] = make_double2(re, im);
}

template <typename C>
__global__ void k_gather_dense(int64_t n, const int64_t* __restrict__ dest, const int64_t* __restrict__ ptr,
                               const int32_t* __restrict__ src, const double2* __restrict__ pool,
                               C* __restrict__ out) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  double re = 0, im = 0;
  for (int64_t j = ptr[k]; j < ptr[k + 1]; ++j) {
    double2 v = pool[src[j]];
    re += v.x;
    im += v.y;
  }
  out[dest[k]] = from_c128<C>(make_double2(re, im));
}

template <typename C>
__device__ inline C zero_value() {
  C z;
  z.x = 0;
  z.y = 0;
  return z;
}
template <>
__device__ inline float zero_value<float>() {
  return 0.f;
}

template <typename C>
__global__ void k_fill_zero(int64_t n, C* __restrict__ out) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += stride) out[k] = zero_value<C>();
}

// Zeroes the entries of the dense subdomain matrices that a completed banded
// factorisation can have left non-zero, 64x64 tiles of the factor layout:
// for each panel p, row tiles p .. ext_l[p] of its column block (the diagonal
// block and L) and column tiles p+1 .. ext_u[p] of its row block (U). The
// extents are those the factorisation recorded by scanning its own data, and
// nothing outside them is non-zero afterwards, so this returns the storage to
// all zeros while writing only the band. One workgroup per (panel, subdomain).
template <typename C>
__global__ void __launch_bounds__(256) k_clear_envelope(const int32_t* __restrict__ Npad,
                                                        const int64_t* __restrict__ mat_off, int np,
                                                        const int32_t* __restrict__ ext_l,
                                                        const int32_t* __restrict__ ext_u, C* __restrict__ A) {
  constexpr int T = 64;
  const int s = blockIdx.y, p = blockIdx.x;
  const int N = Npad[s];
  const int nt = N / T;
  if (p >= nt) return;
  C* M = A + mat_off[s];
  const int el = min(max(ext_l[(int64_t)s * np + p], p), nt - 1);
  const int eu = min(max(ext_u[(int64_t)s * np + p], p), nt - 1);
  const C z = zero_value<C>();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int r = T * p + w; r < T * (el + 1); r += 4) M[(int64_t)r * N + T * p + lane] = z;
  for (int r = T * p + w; r < T * (p + 1); r += 4)
    for (int col = T * (p + 1) + lane; col < T * (eu + 1); col += 64) M[(int64_t)r * N + col] = z;
}

// identity on the padded diagonal part of each dense subdomain matrix
template <typename C>
__global__ void k_pad_identity(int32_t nsub, const int64_t* __restrict__ dof_ptr, const int32_t* __restrict__ Npad,
                               const int64_t* __restrict__ mat_off, C* __restrict__ A) {
  int32_t s = blockIdx.x;
  if (s >= nsub) return;
  int64_t n = dof_ptr[s + 1] - dof_ptr[s];
  int64_t N = Npad[s];
  for (int64_t r = n + threadIdx.x; r < N; r += blockDim.x) {
    C one;
    one.x = 1;
    one.y = 0;
    A[mat_off[s] + r * N + r] = one;
  }
}

// Y = A X, X and Y DOF-major [n][nrhs]; TPR threads per row, each handling
// right-hand sides j = lane, lane + TPR, ...  Workgroups are dealt to the 8
// XCDs round-robin; the grid is a multiple of 8 and workgroup b takes row
// block (b % 8) * (grid / 8) + b / 8, so each XCD sweeps one contiguous band
// of rows and the X rows its band gathers stay in that XCD's own L2.
template <int TPR>
__global__ void __launch_bounds__(256) k_spmm(int64_t nrows, const int64_t* __restrict__ rp,
                                              const int32_t* __restrict__ col, const double2* __restrict__ val,
                                              const double2* __restrict__ X, double2* __restrict__ Y, int nrhs) {
  const int RPB = 256 / TPR;
  const int64_t per = gridDim.x / 8;
  const int64_t blk = (blockIdx.x % 8) * per + blockIdx.x / 8;
  int64_t row = blk * RPB + threadIdx.x / TPR;
  int lane = threadIdx.x % TPR;
  if (row >= nrows) return;
  const int64_t k0 = rp[row], k1 = rp[row + 1];
  for (int j = lane; j < nrhs; j += TPR) {
    double re = 0, im = 0;
    int64_t k = k0;
    // four non-zeros per iteration: all loads issued before the arithmetic
    for (; k + 4 <= k1; k += 4) {
      double2 a[4], x[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = val[k + q];
#pragma unroll
      for (int q = 0; q < 4; ++q) x[q] = X[(int64_t)col[k + q] * nrhs + j];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        re += a[q].x * x[q].x - a[q].y * x[q].y;
        im += a[q].x * x[q].y + a[q].y * x[q].x;
      }
    }
    for (; k < k1; ++k) {
      double2 a = val[k];
      double2 x = X[(int64_t)col[k] * nrhs + j];
      re += a.x * x.x - a.y * x.y;
      im += a.x * x.y + a.y * x.x;
    }
    Y[row * nrhs + j] = make_double2(re, im);
  }
}

// Y = A X for nrhs <= 32, 32 lanes per row (lane j: right-hand side j). The
// row's column indices and values are loaded once, one entry per lane, and
// handed to all 32 lanes with cross-lane shuffles, so that each lane issues
// only the X loads (four in flight). Same XCD row-band mapping as k_spmm.
template <int UNR>
__global__ void __launch_bounds__(256) k_spmm_bcast(int64_t nrows, const int64_t* __restrict__ rp,
                                                    const int32_t* __restrict__ col,
                                                    const double2* __restrict__ val,
                                                    const double2* __restrict__ X, double2* __restrict__ Y,
                                                    int nrhs) {
  const int64_t per = gridDim.x / 8;
  const int64_t blk = (blockIdx.x % 8) * per + blockIdx.x / 8;
  const int64_t row = blk * 8 + threadIdx.x / 32;
  const int lane = threadIdx.x % 32;
  const int half = threadIdx.x & 32;  // first lane of this row's group within the wave
  if (row >= nrows) return;
  const int64_t k0 = rp[row], k1 = rp[row + 1];
  // lanes beyond nrhs read a copy of the last column; entries beyond the row's
  // end read the row's own X row with value zero (no per-entry branches)
  const uint32_t jc = (uint32_t)min(lane, nrhs - 1);
  double re = 0, im = 0;
  for (int64_t kb = k0; kb < k1; kb += 32) {
    const int cnt = (int)min((int64_t)32, k1 - kb);
    int c = (int)row;
    double2 a = make_double2(0.0, 0.0);
    if (lane < cnt) {
      c = col[kb + lane];
      a = val[kb + lane];
    }
    for (int q = 0; q < cnt; q += UNR) {
      double2 x[UNR], aa[UNR];
      uint32_t off[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int src = half + q + u;
        off[u] = (uint32_t)__shfl(c, src, 64) * (uint32_t)nrhs + jc;
        aa[u].x = __shfl(a.x, src, 64);
        aa[u].y = __shfl(a.y, src, 64);
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) x[u] = X[off[u]];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        re = fma(aa[u].x, x[u].x, re);
        re = fma(-aa[u].y, x[u].y, re);
        im = fma(aa[u].x, x[u].y, im);
        im = fma(aa[u].y, x[u].x, im);
      }
    }
  }
  if (lane < nrhs) Y[row * nrhs + lane] = make_double2(re, im);
}

// Y = A X for nrhs <= 64 / NS, one wavefront per row: lane s * W + j
// (W = 64 / NS) takes right-hand side j and entry stream s (entries k0 + s,
// k0 + s + NS, ...). The row index is wave-uniform, so the column indices and
// values come through scalar loads and reach the lanes as SGPR operands (a
// select between the NS streams' values); no cross-lane shuffles except the
// NS-way sum at the end of the row. Four rows per workgroup, XCD bands as in
// k_spmm.
// One chunk of a row held one entry per lane of the row's WD-lane group
// (window position lc, value a): the entries are broadcast by shuffles and the
// X values read from the LDS window, four in flight. Slots beyond cnt take
// the value zero (their lanes hold zero) and read the X row of the chunk's
// last entry, a column the row has.
template <int WD>
__device__ inline void win_chunk(int cnt, int lc, double2 a, const double2* win, int lane, double& re,
                                 double& im) {
  for (int q = 0; q < cnt; q += 4) {
    double2 x[4], aa[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int l = __shfl(lc, min(q + u, cnt - 1), WD);
      aa[u].x = __shfl(a.x, q + u, WD);
      aa[u].y = __shfl(a.y, q + u, WD);
      x[u] = win[l * WD + lane];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      re = fma(aa[u].x, x[u].x, re);
      re = fma(-aa[u].y, x[u].y, re);
      im = fma(aa[u].x, x[u].y, im);
      im = fma(aa[u].y, x[u].x, im);
    }
  }
}

// Y = A X with X staged in LDS per slice of rows (column windows). The rows
// are cut into slices of at most 32 consecutive rows whose non-zeros touch at
// most 128 distinct columns. Workgroup (slice, h) copies those X rows,
// right-hand sides WD h .. WD h + WD - 1, into LDS once (16 WD bytes per row;
// launched with WD = 16: 32 KB per workgroup, five per compute unit; WD = 32
// needs 64 KB, two per compute unit, and measured slower), then forms the
// slice's rows from LDS: WD lanes per row (lane j: right-hand side WD h + j),
// 32 / G rows per WD-lane group (G = 256 / WD groups), the first 32 entries
// of each row loaded before the barrier together with the window. Workgroups
// are dealt to the XCDs in contiguous bands as in k_spmm; the nh
// right-hand-side blocks of a slice are adjacent.
template <int WD>
__global__ void __launch_bounds__(256) k_spmm_win(int32_t nsl, int nh, const int32_t* __restrict__ srow,
                                                  const int32_t* __restrict__ scp, const int32_t* __restrict__ ucol,
                                                  const int64_t* __restrict__ rp, const uint8_t* __restrict__ lcol,
                                                  const double2* __restrict__ val, const double2* __restrict__ X,
                                                  double2* __restrict__ Y, int nrhs) {
  constexpr int G = 256 / WD, CAP = kSpmmWinCap, PASSES = CAP / G, RPG = kSpmmWinRows / G, CH = 32 / WD;
  __shared__ double2 win[CAP * WD];
  const int64_t per = gridDim.x / 8;
  const int64_t b = (blockIdx.x % 8) * per + blockIdx.x / 8;
  const int64_t s = b / nh;
  if (s >= nsl) return;
  const int h = (int)(b % nh);
  const int g = threadIdx.x / WD, lane = threadIdx.x % WD;
  const int j = h * WD + lane;
  const int jc = min(j, nrhs - 1);  // lanes beyond nrhs carry a copy of the last column
  const int c0 = scp[s], U = scp[s + 1] - c0;
  const int row0 = srow[s], nr = srow[s + 1] - row0;
  double2 t[PASSES];
#pragma unroll
  for (int u = 0; u < PASSES; ++u) {
    const int r = g + G * u;
    t[u] = make_double2(0.0, 0.0);
    if (r < U) t[u] = X[(int64_t)ucol[c0 + r] * nrhs + jc];
  }
  // rows g, g + G, ... of the slice: entries lane, WD + lane, ... (first 32)
  int64_t k0[RPG], k1[RPG];
  int lc[RPG][CH];
  double2 a[RPG][CH];
#pragma unroll
  for (int w = 0; w < RPG; ++w) {
    const int rr = g + G * w;
    k0[w] = k1[w] = 0;
    if (rr < nr) {
      k0[w] = rp[row0 + rr];
      k1[w] = rp[row0 + rr + 1];
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int64_t k = k0[w] + WD * c + lane;
      lc[w][c] = 0;
      a[w][c] = make_double2(0.0, 0.0);
      if (k < k1[w]) {
        lc[w][c] = lcol[k];
        a[w][c] = val[k];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < PASSES; ++u) {
    const int r = g + G * u;
    if (r < U) win[r * WD + lane] = t[u];
  }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < RPG; ++w) {
    const int rr = g + G * w;
    if (rr >= nr) break;
    const int64_t n = k1[w] - k0[w];
    double re = 0, im = 0;
#pragma unroll
    for (int c = 0; c < CH; ++c)
      if (n > WD * c) win_chunk<WD>((int)min(n - WD * c, (int64_t)WD), lc[w][c], a[w][c], win, lane, re, im);
    for (int64_t kb = k0[w] + 32; kb < k1[w]; kb += WD) {  // rows with more than 32 entries
      int l = 0;
      double2 v = make_double2(0.0, 0.0);
      if (kb + lane < k1[w]) {
        l = lcol[kb + lane];
        v = val[kb + lane];
      }
      win_chunk<WD>((int)min(k1[w] - kb, (int64_t)WD), l, v, win, lane, re, im);
    }
    if (j < nrhs) Y[(int64_t)(row0 + rr) * nrhs + j] = make_double2(re, im);
  }
}

// xloc[R][j] = v[rowsrc[R]][j] (0 for padded rows), cast to C
template <typename C>
__global__ void k_restrict(int64_t nrows, const int32_t* __restrict__ rowsrc, const double2* __restrict__ v,
                           C* __restrict__ xloc, int nrhs) {
  int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= nrows * nrhs) return;
  int64_t R = idx / nrhs;
  int j = (int)(idx - R * nrhs);
  int32_t e = rowsrc[R];
  double2 x = e >= 0 ? v[(int64_t)e * nrhs + j] : make_double2(0.0, 0.0);
  xloc[idx] = from_c128<C>(x);
}

// z[e][j] = sum_k w[k] zloc[row[k]][j] over the entries k of edge e
// (ptr[e] .. ptr[e+1], in colour order): 32 lanes per edge (lane j: column
// j, then j + 32, ...), eight edges per workgroup; every edge is written
// once, so no clearing pass and no write conflict. Workgroups are dealt to
// the XCDs in contiguous bands of edges as in k_spmm.
template <typename C>
__global__ void __launch_bounds__(256) k_prolong(int64_t ne, const int64_t* __restrict__ ptr,
                                                 const int64_t* __restrict__ row, const double* __restrict__ w,
                                                 const C* __restrict__ zloc, double2* __restrict__ z, int nrhs,
                                                 double2* __restrict__ z2, int64_t ld2) {
  const int64_t per = gridDim.x / 8;
  const int64_t blk = (blockIdx.x % 8) * per + blockIdx.x / 8;
  const int64_t e = blk * 8 + threadIdx.x / 32;
  if (e >= ne) return;
  const int lane = threadIdx.x % 32;
  const int64_t k0 = ptr[e], k1 = ptr[e + 1];
  for (int j = lane; j < nrhs; j += 32) {
    double2 acc = make_double2(0.0, 0.0);
    for (int64_t k = k0; k < k1; ++k) {
      const double2 v = to_c128(zloc[row[k] * nrhs + j]);
      const double wk = w[k];
      acc.x += wk * v.x;
      acc.y += wk * v.y;
    }
    z[e * nrhs + j] = acc;
    if (z2) z2[e * ld2 + j] = acc;
  }
}

// Per tetrahedron: gt[T][n] = k0^2 sum_pq M_{T,n}[p][q] W[p][q] with
// W[p][q] = sum_j lam[e_p][j] u[e_q][j] (transmitter sum of the adjoint and
// forward fields), and rt[T][n] = |T| sum_m (grad l_n . grad l_m) eps_m
// (the P1 stiffness applied to the nodal permittivity).
__global__ void k_grad_tet(int32_t nt, const int32_t* __restrict__ ts, const double* __restrict__ xyz,
                           const int32_t* __restrict__ t2e, const double2* __restrict__ lam,
                           const double2* __restrict__ u, int nrhs, const double2* __restrict__ eps, double k0sq,
                           double2* __restrict__ gt, double2* __restrict__ rt) {
  int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  int32_t v[4], e[6];
  for (int k = 0; k < 4; ++k) v[k] = ts[4 * (size_t)t + k];
  for (int k = 0; k < 6; ++k) e[k] = t2e[6 * (size_t)t + k];
  double g[4][3];
  double vol = tet_geometry(xyz, v, g);
  double G[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) G[i][j] = dot3(g[i], g[j]);
  double2 W[6][6];
  for (int p = 0; p < 6; ++p)
    for (int q = 0; q < 6; ++q) W[p][q] = make_double2(0.0, 0.0);
  for (int j = 0; j < nrhs; ++j) {
    double2 lv[6], uv[6];
    for (int p = 0; p < 6; ++p) {
      lv[p] = lam[(int64_t)e[p] * nrhs + j];
      uv[p] = u[(int64_t)e[p] * nrhs + j];
    }
    for (int p = 0; p < 6; ++p)
      for (int q = 0; q < 6; ++q) {
        W[p][q].x += lv[p].x * uv[q].x - lv[p].y * uv[q].y;
        W[p][q].y += lv[p].x * uv[q].y + lv[p].y * uv[q].x;
      }
  }
  for (int n = 0; n < 4; ++n) {
    double re = 0, im = 0;
    for (int p = 0; p < 6; ++p) {
      int a = cLE[p][0], b = cLE[p][1];
      for (int q = 0; q < 6; ++q) {
        int c = cLE[q][0], d = cLE[q][1];
        double m = vol * (lll(n, a, c) * G[b][d] - lll(n, a, d) * G[b][c] - lll(n, b, c) * G[a][d] +
                          lll(n, b, d) * G[a][c]);
        re += m * W[p][q].x;
        im += m * W[p][q].y;
      }
    }
    gt[4 * (size_t)t + n] = make_double2(k0sq * re, k0sq * im);
    double kr = 0, ki = 0;
    for (int m = 0; m < 4; ++m) {
      double2 em = eps[v[m]];
      kr += G[n][m] * em.x;
      ki += G[n][m] * em.y;
    }
    rt[4 * (size_t)t + n] = make_double2(vol * kr, vol * ki);
  }
}

// Per vertex n (tetrahedra in ascending order): G_n = sum gt, (K1 eps)_n = sum rt,
// grad_n = conj(G_n) + reg * (K1 eps)_n.
__global__ void k_grad_vertex(int32_t nv, const int64_t* __restrict__ v2t_ptr, const int32_t* __restrict__ v2t,
                              const int32_t* __restrict__ ts, const double2* __restrict__ gt,
                              const double2* __restrict__ rt, double reg, double2* __restrict__ grad,
                              double2* __restrict__ keps) {
  int32_t n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nv) return;
  double gr = 0, gi = 0, kr = 0, ki = 0;
  for (int64_t k = v2t_ptr[n]; k < v2t_ptr[n + 1]; ++k) {
    int32_t t = v2t[k];
    int loc = 0;
    while (loc < 3 && ts[4 * (size_t)t + loc] != n) ++loc;
    double2 a = gt[4 * (size_t)t + loc], b = rt[4 * (size_t)t + loc];
    gr += a.x;
    gi += a.y;
    kr += b.x;
    ki += b.y;
  }
  grad[n] = make_double2(gr + reg * kr, -gi + reg * ki);
  keps[n] = make_double2(kr, ki);
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

void launch_grad_tet(hipStream_t s, int32_t nt, const int32_t* ts, const double* xyz, const int32_t* t2e,
                     const double2* lam, const double2* u, int nrhs, const double2* eps, double k0sq, double2* gt,
                     double2* rt) {
  if (nt > 0)
    hipLaunchKernelGGL(k_grad_tet, dim3(nblk(nt, 128)), dim3(128), 0, s, nt, ts, xyz, t2e, lam, u, nrhs, eps, k0sq,
                       gt, rt);
}
void launch_grad_vertex(hipStream_t s, int32_t nv, const int64_t* v2t_ptr, const int32_t* v2t, const int32_t* ts,
                        const double2* gt, const double2* rt, double reg, double2* grad, double2* keps) {
  if (nv > 0)
    hipLaunchKernelGGL(k_grad_vertex, dim3(nblk(nv, 256)), dim3(256), 0, s, nv, v2t_ptr, v2t, ts, gt, rt, reg, grad,
                       keps);
}

void launch_element(hipStream_t s, int32_t nt, const int32_t* ts, const double* xyz, const double2* eps,
                    int eps_kind, double k0sq, double2* out) {
  if (nt > 0) hipLaunchKernelGGL(k_element, dim3(nblk(nt, 128)), dim3(128), 0, s, nt, ts, xyz, eps, eps_kind, k0sq, out);
}
void launch_face(hipStream_t s, int32_t n, const int32_t* ftet, const int32_t* flf, const int32_t* ts,
                 const double* xyz, const double2* eps, int eps_kind, int per_tet_k, double k0, double2 kconst,
                 double2* out, const double2* kface) {
  if (n > 0)
    hipLaunchKernelGGL(k_face, dim3(nblk(n, 128)), dim3(128), 0, s, n, ftet, flf, ts, xyz, eps, eps_kind,
                       per_tet_k, k0, kconst, kface, out);
}
void launch_pec_csr(hipStream_t s, int64_t n, const int64_t* rp, const int32_t* col, const int32_t* pec,
                    double2* val) {
  if (n > 0) hipLaunchKernelGGL(k_pec_csr, dim3(nblk(n, 256)), dim3(256), 0, s, n, rp, col, pec, val);
}
template <typename C>
void launch_pec_local(hipStream_t s, int32_t nsub, const int32_t* Npad, const int64_t* mat_off, const int64_t* ptr,
                      const int32_t* idx, C* A) {
  if (nsub > 0) hipLaunchKernelGGL(k_pec_local<C>, dim3(nsub), dim3(256), 0, s, nsub, Npad, mat_off, ptr, idx, A);
}
template void launch_pec_local<float2>(hipStream_t, int32_t, const int32_t*, const int64_t*, const int64_t*,
                                       const int32_t*, float2*);
template void launch_pec_local<double2>(hipStream_t, int32_t, const int32_t*, const int64_t*, const int64_t*,
                                        const int32_t*, double2*);
void launch_zero_rows(hipStream_t s, int64_t n, const int32_t* rows, int nrhs, double2* B) {
  if (n > 0 && nrhs > 0)
    hipLaunchKernelGGL(k_zero_rows, dim3(nblk(n * nrhs, 256)), dim3(256), 0, s, n, rows, nrhs, B);
}
void launch_gather_csr(hipStream_t s, int64_t n, const int64_t* ptr, const int32_t* src, const double2* pool,
                       double2* out) {
  if (n > 0) hipLaunchKernelGGL(k_gather_csr, dim3(nblk(n, 256)), dim3(256), 0, s, n, ptr, src, pool, out);
}
template <typename C>
void launch_gather_dense(hipStream_t s, int64_t n, const int64_t* dest, const int64_t* ptr, const int32_t* src,
                         const double2* pool, C* out) {
  if (n > 0)
    hipLaunchKernelGGL(k_gather_dense<C>, dim3(nblk(n, 256)), dim3(256), 0, s, n, dest, ptr, src, pool, out);
}
template void launch_gather_dense<float2>(hipStream_t, int64_t, const int64_t*, const int64_t*, const int32_t*,
                                          const double2*, float2*);
template void launch_gather_dense<double2>(hipStream_t, int64_t, const int64_t*, const int64_t*, const int32_t*,
                                           const double2*, double2*);
template <typename C>
void launch_fill_zero(hipStream_t s, int64_t n, C* out) {
  if (n > 0) hipLaunchKernelGGL(k_fill_zero<C>, dim3(4096), dim3(256), 0, s, n, out);
}
template void launch_fill_zero<float2>(hipStream_t, int64_t, float2*);
template void launch_fill_zero<double2>(hipStream_t, int64_t, double2*);
template void launch_fill_zero<float>(hipStream_t, int64_t, float*);
template <typename C>
void launch_clear_envelope(hipStream_t s, int32_t nsub, int np, const int32_t* Npad, const int64_t* mat_off,
                           const int32_t* ext_l, const int32_t* ext_u, C* A) {
  if (nsub > 0 && np > 0)
    hipLaunchKernelGGL(k_clear_envelope<C>, dim3(np, nsub), dim3(256), 0, s, Npad, mat_off, np, ext_l, ext_u, A);
}
template void launch_clear_envelope<float2>(hipStream_t, int32_t, int, const int32_t*, const int64_t*,
                                            const int32_t*, const int32_t*, float2*);
template void launch_clear_envelope<double2>(hipStream_t, int32_t, int, const int32_t*, const int64_t*,
                                             const int32_t*, const int32_t*, double2*);
template <typename C>
void launch_pad_identity(hipStream_t s, int32_t nsub, const int64_t* dof_ptr, const int32_t* Npad,
                         const int64_t* mat_off, C* A) {
  if (nsub > 0) hipLaunchKernelGGL(k_pad_identity<C>, dim3(nsub), dim3(64), 0, s, nsub, dof_ptr, Npad, mat_off, A);
}
template void launch_pad_identity<float2>(hipStream_t, int32_t, const int64_t*, const int32_t*, const int64_t*, float2*);
template void launch_pad_identity<double2>(hipStream_t, int32_t, const int64_t*, const int32_t*, const int64_t*, double2*);

// workgroup count rounded up to a multiple of the XCD count
static inline unsigned nblk8(int64_t n, int64_t per) { return (unsigned)((nblk(n, per) + 7) / 8 * 8); }

void launch_spmm(hipStream_t s, int64_t nrows, const int64_t* rp, const int32_t* col, const double2* val,
                 const double2* X, double2* Y, int nrhs, int variant, const SpmmWindows* win) {
  if (nrows <= 0) return;
  if (variant == 2 && win && win->nsl > 0) {
    const int nh = (nrhs + 15) / 16;
    hipLaunchKernelGGL(k_spmm_win<16>, dim3(nblk8((int64_t)win->nsl * nh, 1)), dim3(256), 0, s, win->nsl, nh,
                       win->srow, win->scp, win->ucol, rp, win->lcol, val, X, Y, nrhs);
  } else if (variant == 1 && nrhs <= 32)
    hipLaunchKernelGGL(k_spmm_bcast<4>, dim3(nblk8(nrows, 8)), dim3(256), 0, s, nrows, rp, col, val, X, Y, nrhs);
  else if (nrhs <= 8)
    hipLaunchKernelGGL(k_spmm<8>, dim3(nblk8(nrows, 32)), dim3(256), 0, s, nrows, rp, col, val, X, Y, nrhs);
  else if (nrhs <= 16)
    hipLaunchKernelGGL(k_spmm<16>, dim3(nblk8(nrows, 16)), dim3(256), 0, s, nrows, rp, col, val, X, Y, nrhs);
  else if (nrhs <= 32)
    hipLaunchKernelGGL(k_spmm<32>, dim3(nblk8(nrows, 8)), dim3(256), 0, s, nrows, rp, col, val, X, Y, nrhs);
  else
    hipLaunchKernelGGL(k_spmm<64>, dim3(nblk8(nrows, 4)), dim3(256), 0, s, nrows, rp, col, val, X, Y, nrhs);
}

template <typename C>
void launch_restrict(hipStream_t s, int64_t nrows, const int32_t* rowsrc, const double2* v, C* xloc, int nrhs) {
  int64_t n = nrows * nrhs;
  if (n > 0) hipLaunchKernelGGL(k_restrict<C>, dim3(nblk(n, 256)), dim3(256), 0, s, nrows, rowsrc, v, xloc, nrhs);
}
template void launch_restrict<float2>(hipStream_t, int64_t, const int32_t*, const double2*, float2*, int);
template void launch_restrict<double2>(hipStream_t, int64_t, const int32_t*, const double2*, double2*, int);

template <typename C>
void launch_prolong(hipStream_t s, int64_t ne, const int64_t* ptr, const int64_t* row, const double* w,
                    const C* zloc, double2* z, int nrhs, double2* z2, int64_t ld2) {
  if (ne > 0)
    hipLaunchKernelGGL(k_prolong<C>, dim3(nblk8(ne, 8)), dim3(256), 0, s, ne, ptr, row, w, zloc, z, nrhs, z2, ld2);
}
template void launch_prolong<float2>(hipStream_t, int64_t, const int64_t*, const int64_t*, const double*,
                                     const float2*, double2*, int, double2*, int64_t);
template void launch_prolong<double2>(hipStream_t, int64_t, const int64_t*, const int64_t*, const double*,
                                      const double2*, double2*, int, double2*, int64_t);

}  // namespace mx
