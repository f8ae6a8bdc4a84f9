// Device-side helpers shared by the gfx950 kernels: complex arithmetic on
// interleaved (re, im) pairs and the 16x16x4 matrix-core (MFMA) instructions.
//
// Lane layouts of v_mfma_{f32,f64}_16x16x4 (64 lanes), checked on gfx950:
//   A operand (16 x 4):  lane l holds A[l % 16][l / 16]
//   B operand (4 x 16):  lane l holds B[l / 16][l % 16]
//   C/D f32  (16 x 16):  lane l, register r holds C[4 * (l / 16) + r][l % 16]
//   C/D f64  (16 x 16):  lane l, register r holds C[l / 16 + 4 * r][l % 16]
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace mx {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename R> struct cplx_t;
template <> struct cplx_t<float> { typedef float2 type; typedef f32x4 acc; };
template <> struct cplx_t<double> { typedef double2 type; typedef f64x4 acc; };

template <typename R> using C_t = typename cplx_t<R>::type;
template <typename R> using Acc_t = typename cplx_t<R>::acc;

template <typename C> __device__ __host__ inline C cmk(decltype(C().x) re, decltype(C().x) im) {
  C z; z.x = re; z.y = im; return z;
}
__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ inline double2 cmulc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
template <typename C> __device__ inline C cdiv(C a, C b) {
  // Smith's algorithm
  typedef decltype(a.x) R;
  C q;
  if (fabs(b.x) >= fabs(b.y)) {
    R r = b.y / b.x, d = b.x + b.y * r;
    q.x = (a.x + a.y * r) / d;
    q.y = (a.y - a.x * r) / d;
  } else {
    R r = b.x / b.y, d = b.y + b.x * r;
    q.x = (a.x * r + a.y) / d;
    q.y = (a.y * r - a.x) / d;
  }
  return q;
}
template <typename C> __device__ inline auto cabs1(C a) -> decltype(a.x) { return fabs(a.x) + fabs(a.y); }

__device__ inline double2 to_c128(float2 a) { return make_double2(a.x, a.y); }
__device__ inline double2 to_c128(double2 a) { return a; }
template <typename C> __device__ inline C from_c128(double2 a);
template <> __device__ inline double2 from_c128<double2>(double2 a) { return a; }
template <> __device__ inline float2 from_c128<float2>(double2 a) { return make_float2((float)a.x, (float)a.y); }

// One 16x16x4 real MFMA step.
__device__ inline f32x4 mfma(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline f64x4 mfma(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Row (within a 16x16 tile) of accumulator register r in lane l.
template <typename R> __device__ inline int acc_row(int lane, int r);
template <> __device__ inline int acc_row<float>(int lane, int r) { return 4 * (lane >> 4) + r; }
template <> __device__ inline int acc_row<double>(int lane, int r) { return (lane >> 4) + 4 * r; }

// Complex 16x16 accumulator: C += A * B with A (16x4) and B (4x16) complex.
// sgn = +1 accumulates A*B, sgn = -1 accumulates -A*B.
template <typename R>
__device__ inline void cmfma(C_t<R> a, C_t<R> b, Acc_t<R>& cre, Acc_t<R>& cim) {
  cre = mfma(a.x, b.x, cre);
  cre = mfma(-a.y, b.y, cre);
  cim = mfma(a.x, b.y, cim);
  cim = mfma(a.y, b.x, cim);
}

// Same product with the sign carried by B's imaginary part: for a B value
// shared by several A tiles the negation is done once per B value.
template <typename R>
__device__ inline void cmfma_nb(C_t<R> a, C_t<R> b, C_t<R> bneg_im, Acc_t<R>& cre, Acc_t<R>& cim) {
  cre = mfma(a.x, b.x, cre);
  cre = mfma(a.y, bneg_im.y, cre);
  cim = mfma(a.x, b.y, cim);
  cim = mfma(a.y, b.x, cim);
}

__device__ inline int lane_id() { return threadIdx.x & 63; }

}  // namespace mx

#define MX_HIP_CHECK(expr)                                                  \
  do {                                                                      \
    hipError_t _e = (expr);                                                 \
    if (_e != hipSuccess) return ::mx::hip_fail(_e, #expr, __FILE__, __LINE__); \
  } while (0)
