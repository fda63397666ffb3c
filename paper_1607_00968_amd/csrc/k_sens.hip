// k_sens.hip -- kernels of the adjoint solve, the sensitivity products of
// full waveform inversion (the Helmholtz forward problem and its
// sensitivities, eq:fwisens) and the 16-bit storage of fields.
//
// With H u = q and H = -Lap_h - omega^2 diag(m (1 - i gamma)),
// dH/dm = -omega^2 diag(1 - i gamma), so for a real model perturbation dm
//   J dm  = omega^2 H^-1 ((1 - i gamma) u . dm)
//   J^H w = omega^2 conj((1 - i gamma) u) . H^-H w,
// and H^-H w = conj(H^-1 conj(w)) because H is complex symmetric.
// Fields u, right-hand sides and results are in the ABI layout [nrhs][N]
// (each source contiguous). 16-bit fields: per source, u / s_c in IEEE half
// precision (re, im), s_c = the source's largest |re| or |im| in FP64; the
// value is formed in FP64, rounded to FP32 and then to FP16 (nearest even).
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace helm {

// dS = omega^2 (1 - i gamma) per unknown.
__global__ void k_sens_coef(int64_t N, const double* __restrict__ gamma, double w2, c128* __restrict__ dS) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) dS[i] = c128{w2, -w2 * gamma[i]};
}
void launch_sens_coef(int64_t N, const double* gamma, double omega, c128* dS, hipStream_t s) {
  hipLaunchKernelGGL(k_sens_coef, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, gamma, omega * omega, dS);
}

// A field value from c128 storage or from its 16-bit storage and scale.
__device__ inline c128 field_at(const c128* U, const __half2* U16, const double* sc, int64_t N, int col, int64_t i) {
  if (U) return U[(int64_t)col * N + i];
  const __half2 h = U16[(int64_t)col * N + i];
  const double s = sc[col];
  return c128{s * (double)__low2float(h), s * (double)__high2float(h)};
}

// out[s][i] = dS[i] u_s[i] dm[i]
__global__ void k_jvp_rhs(int64_t N, int nrhs, const c128* __restrict__ dS, const c128* __restrict__ U,
                          const __half2* __restrict__ U16, const double* __restrict__ sc,
                          const double* __restrict__ dm, c128* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * nrhs) return;
  const int col = (int)(t / N);
  const int64_t i = t - (int64_t)col * N;
  const c128 u = field_at(U, U16, sc, N, col, i), d = dS[i];
  const double a = dm[i];
  out[t] = c128{a * (d.re * u.re - d.im * u.im), a * (d.re * u.im + d.im * u.re)};
}
void launch_jvp_rhs(int64_t N, int nrhs, const c128* dS, const void* U, const void* U16, const double* sc,
                    const double* dm, c128* out, hipStream_t s) {
  const int64_t n = N * nrhs;
  hipLaunchKernelGGL(k_jvp_rhs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, N, nrhs, dS, (const c128*)U,
                     (const __half2*)U16, sc, dm, out);
}

// g[i] = Re sum_s conj(dS[i] u_s[i]) y_s[i], the sources summed in order.
__global__ void k_jtvp_accum(int64_t N, int nrhs, const c128* __restrict__ dS, const c128* __restrict__ U,
                             const __half2* __restrict__ U16, const double* __restrict__ sc,
                             const c128* __restrict__ Y, double* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const c128 d = dS[i];
  double acc = 0.0;
  for (int col = 0; col < nrhs; ++col) {
    const c128 u = field_at(U, U16, sc, N, col, i);
    const double pr = d.re * u.re - d.im * u.im, pi = d.re * u.im + d.im * u.re;  // dS u
    const c128 y = Y[(int64_t)col * N + i];
    acc += pr * y.re + pi * y.im;  // Re(conj(dS u) y)
  }
  g[i] = acc;
}
void launch_jtvp_accum(int64_t N, int nrhs, const c128* dS, const void* U, const void* U16, const double* sc,
                       const c128* Y, double* g, hipStream_t s) {
  hipLaunchKernelGGL(k_jtvp_accum, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, nrhs, dS, (const c128*)U,
                     (const __half2*)U16, sc, Y, g);
}

// x <- conj(x), n complex values.
__global__ void k_conj(int64_t n, c128* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i].im = -x[i].im;
}
void launch_conj(int64_t n, c128* x, hipStream_t s) {
  hipLaunchKernelGGL(k_conj, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, x);
}

// Per-source scale of the 16-bit storage: the largest |re| or |im| of the
// column (1 for a zero column). One workgroup per column.
__global__ __launch_bounds__(256) void k_col_absmax(int64_t N, const c128* __restrict__ U, double* __restrict__ sc) {
  __shared__ double red[256];
  const int col = blockIdx.x;
  const c128* u = U + (int64_t)col * N;
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += 256) m = fmax(m, fmax(fabs(u[i].re), fabs(u[i].im)));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) sc[col] = red[0] > 0.0 ? red[0] : 1.0;
}

__global__ void k_pack16(int64_t N, int nrhs, const c128* __restrict__ U, const double* __restrict__ sc,
                         __half2* __restrict__ H) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * nrhs) return;
  const int col = (int)(t / N);
  const double s = sc[col];
  const c128 u = U[t];
  H[t] = __halves2half2(__float2half_rn((float)(u.re / s)), __float2half_rn((float)(u.im / s)));
}

__global__ void k_unpack16(int64_t N, int nrhs, const __half2* __restrict__ H, const double* __restrict__ sc,
                           c128* __restrict__ U) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * nrhs) return;
  const int col = (int)(t / N);
  const double s = sc[col];
  U[t] = c128{s * (double)__low2float(H[t]), s * (double)__high2float(H[t])};
}

void launch_pack16(int64_t N, int nrhs, const c128* U, double* sc, void* H, hipStream_t s) {
  hipLaunchKernelGGL(k_col_absmax, dim3(nrhs), dim3(256), 0, s, N, U, sc);
  const int64_t n = N * nrhs;
  hipLaunchKernelGGL(k_pack16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, N, nrhs, U, (const double*)sc,
                     (__half2*)H);
}

void launch_unpack16(int64_t N, int nrhs, const void* H, const double* sc, c128* U, hipStream_t s) {
  const int64_t n = N * nrhs;
  hipLaunchKernelGGL(k_unpack16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, N, nrhs, (const __half2*)H, sc,
                     U);
}

}  // namespace helm
