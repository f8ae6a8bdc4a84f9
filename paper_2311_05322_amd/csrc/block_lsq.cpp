// Block FGMRES least squares on the host (declarations and layout in
// block_lsq.h). A cycle of m block steps of width s = 32 applies about
// m^2 s^2 / 2 rotations to rows of s values and ends with a back substitution
// of (m s)^2 s / 2 complex multiply-adds, while the GPU waits; the hot loops
// are therefore written over split real/imaginary rows and built in three
// instruction-set versions (AVX-512, AVX2 + FMA, baseline), the widest one the
// CPU reports being used.
#include "block_lsq.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace mx {

namespace {

typedef std::complex<double> cd;

#define MX_INLINE inline __attribute__((always_inline))

// [a; b] <- [c, sn; -conj(sn), c] [a; b] on n values of two split rows
MX_INLINE void rot_rows(double* __restrict ar, double* __restrict ai, double* __restrict br, double* __restrict bi,
                     int n, double c, double sr, double si) {
  for (int q = 0; q < n; ++q) {
    const double xr = ar[q], xi = ai[q], yr = br[q], yi = bi[q];
    ar[q] = c * xr + sr * yr - si * yi;
    ai[q] = c * xi + sr * yi + si * yr;
    br[q] = c * yr - sr * xr - si * xi;
    bi[q] = c * yi - sr * xi + si * xr;
  }
}

// rotations u = 0 .. cnt-1 of row cc against rows rj[u] in turn (one column
// of a triangularised block: row cc is held in registers over the fan; S > 0
// fixes the row length at compile time)
template <int S>
MX_INLINE void rot_fan(double* pr, double* pi, int s_rt, int32_t cc, const int32_t* rj, const double* rc,
                       const double* rsr, const double* rsi, size_t cnt) {
  const int s = S > 0 ? S : s_rt;
  double xr[32], xi[32];
  double* ar = pr + (size_t)cc * s;
  double* ai = pi + (size_t)cc * s;
  for (int q = 0; q < s; ++q) {
    xr[q] = ar[q];
    xi[q] = ai[q];
  }
  for (size_t u = 0; u < cnt; ++u) {
    double* __restrict br = pr + (size_t)rj[u] * s;
    double* __restrict bi = pi + (size_t)rj[u] * s;
    const double c = rc[u], sr = rsr[u], si = rsi[u];
    for (int q = 0; q < s; ++q) {
      const double x0 = xr[q], x1 = xi[q], y0 = br[q], y1 = bi[q];
      xr[q] = c * x0 + sr * y0 - si * y1;
      xi[q] = c * x1 + sr * y1 + si * y0;
      br[q] = c * y0 - sr * x0 - si * x1;
      bi[q] = c * y1 - sr * x1 + si * x0;
    }
  }
  for (int q = 0; q < s; ++q) {
    ar[q] = xr[q];
    ai[q] = xi[q];
  }
}

// the recorded rotations [0, nrot) on the rows of a block column (stride
// s <= 32), in order; consecutive rotations share their first row
MX_INLINE void rot_list_body(double* pr, double* pi, int s, size_t nrot, const int32_t* ri, const int32_t* rj,
                             const double* rc, const double* rsr, const double* rsi) {
  size_t t = 0;
  while (t < nrot) {
    size_t t1 = t + 1;
    while (t1 < nrot && ri[t1] == ri[t]) ++t1;
    if (s == 32)
      rot_fan<32>(pr, pi, s, ri[t], rj + t, rc + t, rsr + t, rsi + t, t1 - t);
    else
      rot_fan<0>(pr, pi, s, ri[t], rj + t, rc + t, rsr + t, rsi + t, t1 - t);
    t = t1;
  }
}

// zeroes the sub-diagonal part of block column k (rows k s + jj + 1 ..
// (k+1) s + jj of its column jj, one rotation each against the diagonal row),
// rotating the right-hand sides along; the rotations are appended
MX_INLINE void triangularise_body(double* pr, double* pi, double* gr, double* gi, int s, int k, int32_t* ri,
                                 int32_t* rj, double* rc, double* rsr, double* rsi) {
  size_t t = 0;
  for (int jj = 0; jj < s; ++jj) {
    const int64_t cc = (int64_t)k * s + jj;
    for (int64_t r = cc + 1; r <= (int64_t)(k + 1) * s + jj; ++r) {
      const cd a(pr[cc * s + jj], pi[cc * s + jj]);
      const cd b(pr[r * s + jj], pi[r * s + jj]);
      double c;
      cd sn;
      if (b == 0.0) {
        c = 1.0;
        sn = 0.0;
      } else if (a == 0.0) {
        c = 0.0;
        sn = std::conj(b) / std::abs(b);
      } else {
        const double den = std::hypot(std::abs(a), std::abs(b));
        c = std::abs(a) / den;
        sn = (a / std::abs(a)) * std::conj(b) / den;
      }
      rot_rows(pr + cc * s + jj, pi + cc * s + jj, pr + r * s + jj, pi + r * s + jj, s - jj, c, sn.real(),
               sn.imag());
      pr[r * s + jj] = pi[r * s + jj] = 0.0;
      rot_rows(gr + cc * s, gi + cc * s, gr + r * s, gi + r * s, s, c, sn.real(), sn.imag());
      ri[t] = (int32_t)cc;
      rj[t] = (int32_t)r;
      rc[t] = c;
      rsr[t] = sn.real();
      rsi[t] = sn.imag();
      ++t;
    }
  }
}

// y [n][s] (split) from the upper triangular H (leading n x n of [.][ncol])
// and the rotated right-hand sides g: row i from rows i+1 .. n-1 (s <= 32;
// S > 0 fixes s at compile time so that the row being solved stays in
// registers)
template <int S>
MX_INLINE void back_subst_rows(const double* hr, const double* hi, int64_t ncol, const double* gr, const double* gi,
                               int64_t n, int s_rt, double* __restrict yr, double* __restrict yi) {
  const int s = S > 0 ? S : s_rt;
  double vr[32], vi[32];
  for (int64_t i = n - 1; i >= 0; --i) {
    for (int q = 0; q < s; ++q) {
      vr[q] = gr[i * s + q];
      vi[q] = gi[i * s + q];
    }
    const double* hri = hr + i * ncol;
    const double* hii = hi + i * ncol;
    for (int64_t j = i + 1; j < n; ++j) {
      const double a = hri[j], b = hii[j];
      const double* yrj = yr + j * s;
      const double* yij = yi + j * s;
      for (int q = 0; q < s; ++q) {
        vr[q] -= a * yrj[q] - b * yij[q];
        vi[q] -= a * yij[q] + b * yrj[q];
      }
    }
    const cd d(hri[i], hii[i]);
    const cd dinv = d != 0.0 ? 1.0 / d : cd(0.0);
    for (int q = 0; q < s; ++q) {
      yr[i * s + q] = dinv.real() * vr[q] - dinv.imag() * vi[q];
      yi[i * s + q] = dinv.real() * vi[q] + dinv.imag() * vr[q];
    }
  }
}

MX_INLINE void back_subst_body(const double* hr, const double* hi, int64_t ncol, const double* gr, const double* gi,
                               int64_t n, int s, double* yr, double* yi) {
  if (s == 32)
    back_subst_rows<32>(hr, hi, ncol, gr, gi, n, s, yr, yi);
  else
    back_subst_rows<0>(hr, hi, ncol, gr, gi, n, s, yr, yi);
}

// one entry per instruction-set version
#define MX_ISA_VERSIONS(NAME, PARAMS, ARGS)                                                                  \
  __attribute__((target("avx512f,avx512dq,avx512vl,avx2,fma"))) void NAME##_v4 PARAMS { NAME##_body ARGS; } \
  __attribute__((target("avx2,fma"))) void NAME##_v3 PARAMS { NAME##_body ARGS; }                           \
  void NAME##_v0 PARAMS { NAME##_body ARGS; }                                                                \
  void NAME PARAMS {                                                                                         \
    const int v = isa_level();                                                                               \
    if (v == 2)                                                                                              \
      NAME##_v4 ARGS;                                                                                        \
    else if (v == 1)                                                                                         \
      NAME##_v3 ARGS;                                                                                        \
    else                                                                                                     \
      NAME##_v0 ARGS;                                                                                        \
  }

// 2: AVX-512 (F, DQ, VL), 1: AVX2 and FMA, 0: neither
int isa_level() {
  static const int v = [] {
    __builtin_cpu_init();
    const bool v3 = __builtin_cpu_supports("avx2") && __builtin_cpu_supports("fma");
    const bool v4 = v3 && __builtin_cpu_supports("avx512f") && __builtin_cpu_supports("avx512dq") &&
                    __builtin_cpu_supports("avx512vl");
    return v4 ? 2 : v3 ? 1 : 0;
  }();
  return v;
}

MX_ISA_VERSIONS(rot_list,
                (double* pr, double* pi, int s, size_t nrot, const int32_t* ri, const int32_t* rj, const double* rc,
                 const double* rsr, const double* rsi),
                (pr, pi, s, nrot, ri, rj, rc, rsr, rsi))
MX_ISA_VERSIONS(triangularise,
                (double* pr, double* pi, double* gr, double* gi, int s, int k, int32_t* ri, int32_t* rj, double* rc,
                 double* rsr, double* rsi),
                (pr, pi, gr, gi, s, k, ri, rj, rc, rsr, rsi))
MX_ISA_VERSIONS(back_subst,
                (const double* hr, const double* hi, int64_t ncol, const double* gr, const double* gi, int64_t n,
                 int s, double* yr, double* yi),
                (hr, hi, ncol, gr, gi, n, s, yr, yi))

}  // namespace

void BlockLsq::reset(int s, int m, const std::vector<cd>& S0) {
  // the register-held rows of the rotations and the back substitution hold 32
  // values (block FGMRES splits wider blocks into groups of at most 32)
  if (s < 1 || s > 32 || m < 1) throw std::invalid_argument("BlockLsq: block width must be 1..32, m >= 1");
  s_ = s;
  m_ = m;
  kdone_ = 0;
  const size_t nrow = (size_t)(m + 1) * s;
  ncol_ = (int64_t)m * s;
  // every entry of the Hessenberg planes that a solve reads is written by add
  hr_.resize(nrow * ncol_);
  hi_.resize(nrow * ncol_);
  gr_.assign(nrow * s, 0.0);
  gi_.assign(nrow * s, 0.0);
  for (size_t e = 0; e < (size_t)s * s; ++e) {
    gr_[e] = S0[e].real();
    gi_[e] = S0[e].imag();
  }
  pr_.resize(nrow * s);
  pi_.resize(nrow * s);
  const size_t nrot = (size_t)m * s * s;
  ri_.resize(nrot);
  rj_.resize(nrot);
  rc_.resize(nrot);
  rsr_.resize(nrot);
  rsi_.resize(nrot);
}

void BlockLsq::add(int k, const std::vector<cd>& P) {
  const int s = s_;
  const size_t ne = (size_t)(k + 2) * s * s;
  for (size_t e = 0; e < ne; ++e) {
    pr_[e] = P[e].real();
    pi_[e] = P[e].imag();
  }
  // the rotations of the previous block columns (s^2 per column), then this
  // column's own
  const size_t nold = (size_t)k * s * s;
  rot_list(pr_.data(), pi_.data(), s, nold, ri_.data(), rj_.data(), rc_.data(), rsr_.data(), rsi_.data());
  triangularise(pr_.data(), pi_.data(), gr_.data(), gi_.data(), s, k, ri_.data() + nold, rj_.data() + nold,
                rc_.data() + nold, rsr_.data() + nold, rsi_.data() + nold);
  const int64_t rows = (int64_t)(k + 2) * s;
  for (int64_t i = 0; i < rows; ++i)
    for (int q = 0; q < s; ++q) {
      hr_[(size_t)(i * ncol_ + (int64_t)k * s + q)] = pr_[(size_t)i * s + q];
      hi_[(size_t)(i * ncol_ + (int64_t)k * s + q)] = pi_[(size_t)i * s + q];
    }
  kdone_ = k + 1;
}

double BlockLsq::colres(int b) const {
  double t = 0;
  for (int64_t i = (int64_t)kdone_ * s_; i < (int64_t)(kdone_ + 1) * s_; ++i) {
    const double x = gr_[(size_t)i * s_ + b], y = gi_[(size_t)i * s_ + b];
    t += x * x + y * y;
  }
  return std::sqrt(t);
}

void BlockLsq::solve(double* Y) const {
  const int64_t n = (int64_t)kdone_ * s_;
  std::vector<double> yr((size_t)(n * s_)), yi((size_t)(n * s_));
  back_subst(hr_.data(), hi_.data(), ncol_, gr_.data(), gi_.data(), n, s_, yr.data(), yi.data());
  for (size_t e = 0; e < yr.size(); ++e) {
    Y[2 * e] = yr[e];
    Y[2 * e + 1] = yi[e];
  }
}

}  // namespace mx
