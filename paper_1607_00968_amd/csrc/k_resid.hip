// k_resid.hip -- the final FP64 residual check of a block solve (the
// stopping rule of section 5.3: every right-hand side's residual reduced by
// the tolerance), computed straight from the caller's blocks.
//
// relres_s = ||q_s - H u_s||_2 / ||q_s||_2 with H = -Lap_h - omega^2 m (1 - i
// gamma) (eq:helm / eq:LinearSystem). Q and U stay in the ABI layout
// [nrhs][N] (each right-hand side contiguous, grid axis 0 fastest): one pass
// reads them once, forms r in registers and accumulates ||r||^2 and ||q||^2
// per column; nothing of size N is written. The per-workgroup partial sums
// go to a small buffer (at most RESID_MAX_COLS x RESID_MAX_CHUNKS x 2
// doubles) and a second kernel reduces them in a fixed order, so the result
// does not depend on scheduling.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.hpp"

namespace helm {

// Partial sums of helm_residual_noalloc, for callers that cannot allocate:
// the largest block (RESID_MAX_COLS columns x RESID_MAX_CHUNKS chunks x 2
// doubles, plus one result per column), about 1 MB, held by every device the
// library runs on until the process ends. Host code never passes this
// name to a kernel: it is a host-side stand-in, and the device address comes
// from hipGetSymbolAddress, per device, in resid_static_scratch below.
constexpr size_t RESID_STATIC_DOUBLES = (size_t)RESID_MAX_COLS * (2 * RESID_MAX_CHUNKS + 1);
static __device__ __align__(256) double scratch[RESID_STATIC_DOUBLES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t resid_static_scratch(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// (H u)_i for column-contiguous u: dH_i u_i - sum_d ih_d (u_{i-e_d} + u_{i+e_d}),
// zero outside the grid (homogeneous Dirichlet values).
__global__ __launch_bounds__(256) void k_resid_part(int64_t N, int nx, int ny, int nz, int chunks, double ih0,
                                                    double ih1, double ih2, const c128* __restrict__ dH,
                                                    const c128* __restrict__ Q, const c128* __restrict__ U,
                                                    double* __restrict__ part) {
  __shared__ double red[2][256];
  // consecutive workgroups take the same chunk of different columns, so the
  // chunk's diagonal is fetched from HBM about once
  const int col = blockIdx.x;
  const int64_t per = (N + chunks - 1) / chunks;
  const int64_t i0 = (int64_t)blockIdx.y * per;
  const int64_t i1 = i0 + per < N ? i0 + per : N;
  const c128* q = Q + (int64_t)col * N;
  const c128* u = U + (int64_t)col * N;
  const int64_t nxy = (int64_t)nx * ny;
  double r2 = 0.0, q2 = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
    const int x = (int)(i % nx);
    const int y = (int)((i / nx) % ny);
    const int z = (int)(i / nxy);
    const c128 uc = u[i];
    const c128 d = dH[i];
    double hr = d.re * uc.re - d.im * uc.im;
    double hi = d.re * uc.im + d.im * uc.re;
    double sr = 0.0, si = 0.0;
    if (x > 0) { sr += u[i - 1].re; si += u[i - 1].im; }
    if (x < nx - 1) { sr += u[i + 1].re; si += u[i + 1].im; }
    hr -= ih0 * sr;
    hi -= ih0 * si;
    sr = 0.0;
    si = 0.0;
    if (y > 0) { sr += u[i - nx].re; si += u[i - nx].im; }
    if (y < ny - 1) { sr += u[i + nx].re; si += u[i + nx].im; }
    hr -= ih1 * sr;
    hi -= ih1 * si;
    if (nz > 1) {
      sr = 0.0;
      si = 0.0;
      if (z > 0) { sr += u[i - nxy].re; si += u[i - nxy].im; }
      if (z < nz - 1) { sr += u[i + nxy].re; si += u[i + nxy].im; }
      hr -= ih2 * sr;
      hi -= ih2 * si;
    }
    const c128 qc = q[i];
    const double rr = qc.re - hr, ri = qc.im - hi;
    r2 += rr * rr + ri * ri;
    q2 += qc.re * qc.re + qc.im * qc.im;
  }
  red[0][threadIdx.x] = r2;
  red[1][threadIdx.x] = q2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((int64_t)col * chunks + blockIdx.y) * 2 + 0] = red[0][0];
    part[((int64_t)col * chunks + blockIdx.y) * 2 + 1] = red[1][0];
  }
}

// One workgroup per column: fixed-order sum of its `chunks` partials, then
// relres = sqrt(r2 / q2) (0 for a zero right-hand side).
__global__ __launch_bounds__(256) void k_resid_final(int chunks, const double* __restrict__ part,
                                                     double* __restrict__ relres) {
  __shared__ double red[2][256];
  const int col = blockIdx.x;
  double r2 = 0.0, q2 = 0.0;
  for (int b = threadIdx.x; b < chunks; b += 256) {
    r2 += part[((int64_t)col * chunks + b) * 2 + 0];
    q2 += part[((int64_t)col * chunks + b) * 2 + 1];
  }
  red[0][threadIdx.x] = r2;
  red[1][threadIdx.x] = q2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) relres[col] = red[1][0] > 0.0 ? sqrt(red[0][0] / red[1][0]) : 0.0;
}

int resid_chunks(int64_t N) {
  // at least 2048 points (8 per lane) per workgroup, at most RESID_MAX_CHUNKS
  int64_t c = (N + 2047) / 2048;
  if (c > RESID_MAX_CHUNKS) c = RESID_MAX_CHUNKS;
  return c < 1 ? 1 : (int)c;
}

size_t resid_scratch_doubles(int nrhs, int64_t N) { return (size_t)nrhs * resid_chunks(N) * 2 + (size_t)nrhs; }

void launch_resid_norms(const Geo& g, int nrhs, const double ih[3], const c128* dH, const void* Q, const void* U,
                        double* scratch, hipStream_t s) {
  if (nrhs < 1 || nrhs > RESID_MAX_COLS) fatal_combo("launch_resid_norms");
  const int chunks = resid_chunks(g.npts);
  double* part = scratch + nrhs;
  hipLaunchKernelGGL(k_resid_part, dim3(nrhs, chunks), dim3(256), 0, s, g.npts, g.nx, g.ny, g.nz, chunks, ih[0],
                     ih[1], ih[2], dH, (const c128*)Q, (const c128*)U, part);
  hipLaunchKernelGGL(k_resid_final, dim3(nrhs), dim3(256), 0, s, chunks, (const double*)part, scratch);
}

}  // namespace helm
