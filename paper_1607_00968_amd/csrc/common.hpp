// common.hpp -- device-side types shared by the solver's HIP kernels.
//
// Internal field layout: a block of P right-hand sides over N grid points is
// stored point-major, [N][Pp] (Pp = P rounded up to a multiple of 4), so the
// values of every RHS at one point are contiguous. Stencil kernels then read
// one coalesced run per neighbour and load each point's coefficients once
// for the whole block (the block multigrid cycle of the paper: every
// relaxation, restriction and interpolation acts on the block).
//
// Storage types: c128 (2 x fp64), c64 (2 x fp32), cbf (2 x bf16, round to
// nearest even). Each lane moves 16 bytes: 1, 2 or 4 complex values.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace helm {

struct alignas(16) c128 { double re, im; };
struct alignas(8) c64 { float re, im; };
struct alignas(4) cbf { uint16_t re, im; };

template <class T> struct cx { T re, im; };

template <class T> __device__ __host__ inline cx<T> cmk(T r, T i) { return cx<T>{r, i}; }
template <class T> __device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T> __device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T> __device__ inline cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T> __device__ inline cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
// a += b * c
template <class T> __device__ inline void cfma(cx<T>& a, cx<T> b, cx<T> c) {
  a.re = fma(b.re, c.re, a.re);
  a.re = fma(-b.im, c.im, a.re);
  a.im = fma(b.re, c.im, a.im);
  a.im = fma(b.im, c.re, a.im);
}
// a += conj(b) * c
template <class T> __device__ inline void cfmac(cx<T>& a, cx<T> b, cx<T> c) {
  a.re = fma(b.re, c.re, a.re);
  a.re = fma(b.im, c.im, a.re);
  a.im = fma(b.re, c.im, a.im);
  a.im = fma(-b.im, c.re, a.im);
}

// ---- bf16 with round-to-nearest-even ---------------------------------------
__device__ __host__ inline uint16_t f2bf(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __host__ inline float bf2f(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }

// ---- per-lane vectors of R complex values (16 bytes) -----------------------
template <class S> struct St;
template <> struct St<c128> { static constexpr int R = 1; };
template <> struct St<c64> { static constexpr int R = 2; };
template <> struct St<cbf> { static constexpr int R = 4; };

template <class S, class T> struct Vec { cx<T> v[St<S>::R]; };

template <class T> __device__ inline void ld16(const c128* p, cx<T>* o) {
  double2 a = *reinterpret_cast<const double2*>(p);
  o[0] = {(T)a.x, (T)a.y};
}
template <class T> __device__ inline void ld16(const c64* p, cx<T>* o) {
  float4 a = *reinterpret_cast<const float4*>(p);
  o[0] = {(T)a.x, (T)a.y};
  o[1] = {(T)a.z, (T)a.w};
}
template <class T> __device__ inline void ld16(const cbf* p, cx<T>* o) {
  uint4 a = *reinterpret_cast<const uint4*>(p);
  uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) o[k] = {(T)bf2f((uint16_t)(w[k] & 0xffffu)), (T)bf2f((uint16_t)(w[k] >> 16))};
}
template <class T> __device__ inline void st16(c128* p, const cx<T>* o) {
  *reinterpret_cast<double2*>(p) = double2{(double)o[0].re, (double)o[0].im};
}
template <class T> __device__ inline void st16(c64* p, const cx<T>* o) {
  *reinterpret_cast<float4*>(p) = float4{(float)o[0].re, (float)o[0].im, (float)o[1].re, (float)o[1].im};
}
template <class T> __device__ inline void st16(cbf* p, const cx<T>* o) {
  uint32_t w[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) w[k] = (uint32_t)f2bf((float)o[k].re) | ((uint32_t)f2bf((float)o[k].im) << 16);
  *reinterpret_cast<uint4*>(p) = uint4{w[0], w[1], w[2], w[3]};
}

// Load R values, or zeros when `ok` is false (a neighbour outside the grid).
template <class S, class T> __device__ inline void ldz(const S* p, bool ok, cx<T>* o) {
  if (ok) {
    ld16<T>(p, o);
  } else {
#pragma unroll
    for (int k = 0; k < St<S>::R; ++k) o[k] = {(T)0, (T)0};
  }
}

// Coefficient loads (one complex, broadcast to the lanes of a point).
template <class T> __device__ inline cx<T> ldc(const cx<T>* p) { return *p; }

// Level geometry passed by value to kernels.
struct Geo {
  int nx, ny, nz;   // unknowns per axis (nz = 1 in 2D)
  int64_t npts;
  int P;            // padded RHS count per point (multiple of 4)
};

__device__ inline void coords(const Geo& g, int64_t i, int& x, int& y, int& z) {
  x = (int)(i % g.nx);
  int64_t r = i / g.nx;
  y = (int)(r % g.ny);
  z = (int)(r / g.ny);
}

}  // namespace helm
