// Shared device/host helpers for libtransec_gpu (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <string>

namespace tsg {

// Complex numbers as plain structs so that kernels stay free of library
// complex types; T is float (complex64 storage) or double (complex128).
template <typename T> struct alignas(2 * sizeof(T)) cplx { T re, im; };
using c64 = cplx<float>;
using c128 = cplx<double>;

template <typename T> __host__ __device__ inline cplx<T> mk(T r, T i) { return cplx<T>{r, i}; }
template <typename T> __host__ __device__ inline cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __host__ __device__ inline cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __host__ __device__ inline cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __host__ __device__ inline cplx<T> operator*(T s, cplx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> __host__ __device__ inline cplx<T> conj(cplx<T> a) { return {a.re, -a.im}; }
template <typename T> __host__ __device__ inline T norm2(cplx<T> a) { return a.re * a.re + a.im * a.im; }
template <typename T> __host__ __device__ inline T cabs(cplx<T> a) { return sqrt(a.re * a.re + a.im * a.im); }
// a += b * c
template <typename T> __host__ __device__ inline void fma_acc(cplx<T>& a, cplx<T> b, cplx<T> c) {
  a.re = fma(b.re, c.re, a.re); a.re = fma(-b.im, c.im, a.re);
  a.im = fma(b.re, c.im, a.im); a.im = fma(b.im, c.re, a.im);
}
// a += conj(b) * c
template <typename T> __host__ __device__ inline void fma_cacc(cplx<T>& a, cplx<T> b, cplx<T> c) {
  a.re = fma(b.re, c.re, a.re); a.re = fma(b.im, c.im, a.re);
  a.im = fma(b.re, c.im, a.im); a.im = fma(-b.im, c.re, a.im);
}
template <typename T> __host__ __device__ inline cplx<T> cdiv(cplx<T> a, cplx<T> b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    T r = b.im / b.re, d = b.re + r * b.im;
    return {(a.re + r * a.im) / d, (a.im - r * a.re) / d};
  } else {
    T r = b.re / b.im, d = b.im + r * b.re;
    return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
  }
}
template <typename T> __host__ __device__ inline cplx<T> csqrt(cplx<T> z) {
  // principal branch
  T a = cabs(z);
  if (a == T(0)) return {T(0), T(0)};
  T re = sqrt(T(0.5) * (a + fabs(z.re)));
  T im = T(0.5) * z.im / re;
  if (z.re >= T(0)) return {re, im};
  return {fabs(im), z.im >= T(0) ? re : -re};
}

// Element precision codes used across the C-ABI.
enum Precision : int32_t { kFP64 = 0, kFP32Bulk = 1 };

struct Status {
  int code = 0;
  std::string msg;
};

}  // namespace tsg

#define TSG_HIP_CHECK(expr)                                                          \
  do {                                                                               \
    hipError_t _e = (expr);                                                          \
    if (_e != hipSuccess) {                                                          \
      throw ::tsg::DeviceError(std::string(#expr) + ": " + hipGetErrorString(_e)); \
    }                                                                                \
  } while (0)

namespace tsg {
struct DeviceError {
  std::string what;
  explicit DeviceError(std::string w) : what(std::move(w)) {}
};
}  // namespace tsg
