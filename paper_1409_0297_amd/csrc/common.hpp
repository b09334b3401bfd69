// Shared device/host helpers of the HIP library: complex arithmetic on
// interleaved (re, im) pairs, error plumbing, launch helpers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

namespace spp {

// ---------------------------------------------------------------- complex
template <typename R> struct cplx;
template <> struct cplx<double> { using type = double2; };
template <> struct cplx<float> { using type = float2; };
template <typename R> using cplx_t = typename cplx<R>::type;

template <typename C> __host__ __device__ inline C cmake(decltype(C::x) re, decltype(C::x) im) {
  C c; c.x = re; c.y = im; return c;
}
template <typename C> __host__ __device__ inline C cadd(C a, C b) { return cmake<C>(a.x + b.x, a.y + b.y); }
template <typename C> __host__ __device__ inline C csub(C a, C b) { return cmake<C>(a.x - b.x, a.y - b.y); }
template <typename C> __host__ __device__ inline C cneg(C a) { return cmake<C>(-a.x, -a.y); }
template <typename C> __host__ __device__ inline C cmul(C a, C b) {
  return cmake<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C> __host__ __device__ inline C cconjmul(C a, C b) {   // conj(a) * b
  return cmake<C>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <typename C> __host__ __device__ inline C cscale(C a, decltype(C::x) s) { return cmake<C>(a.x * s, a.y * s); }
// acc += a * b
template <typename C> __host__ __device__ inline void cfma(C& acc, C a, C b) {
  acc.x += a.x * b.x - a.y * b.y;
  acc.y += a.x * b.y + a.y * b.x;
}
// acc -= a * b
template <typename C> __host__ __device__ inline void cfms(C& acc, C a, C b) {
  acc.x -= a.x * b.x - a.y * b.y;
  acc.y -= a.x * b.y + a.y * b.x;
}
template <typename C> __host__ __device__ inline decltype(C::x) cabs2(C a) { return a.x * a.x + a.y * a.y; }
template <typename C> __device__ inline C cdiv(C a, C b) {
  using R = decltype(C::x);
  R d = b.x * b.x + b.y * b.y;
  return cmake<C>((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
template <typename C> __device__ inline C crecip(C b) {
  using R = decltype(C::x);
  R d = b.x * b.x + b.y * b.y;
  return cmake<C>(b.x / d, -b.y / d);
}

template <typename Dst, typename Src> __host__ __device__ inline Dst cconvert(Src s) {
  Dst d; d.x = static_cast<decltype(Dst::x)>(s.x); d.y = static_cast<decltype(Dst::x)>(s.y); return d;
}

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void throw_hip(hipError_t e, const char* what, const char* file, int line);

#define SPP_HIP(call)                                                   \
  do {                                                                  \
    hipError_t _e = (call);                                             \
    if (_e != hipSuccess) ::spp::throw_hip(_e, #call, __FILE__, __LINE__); \
  } while (0)

#define SPP_LAUNCH_CHECK() SPP_HIP(hipGetLastError())

inline unsigned ceil_div(int64_t a, int64_t b) { return static_cast<unsigned>((a + b - 1) / b); }

}  // namespace spp
