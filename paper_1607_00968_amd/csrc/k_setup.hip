// k_setup.hip -- hierarchy construction (setup, not on the per-solve path)
// and the dense complex GEMM used by the coarsest-grid solve.
//
//  - fine diagonals of H and of the shifted M (eq:helm, eq:LinearSystem; the
//    shift adds a positive constant to gamma);
//  - Galerkin coarse operators R M P with d-linear P and R = 2^-d P^T,
//    computed directly in stencil form: each 3^d coarse stencil entry is the
//    sum over the fine couplings that connect the supports of the two coarse
//    basis functions;
//  - the coarsest operator assembled densely and inverted in FP64 by blocked
//    Gauss-Jordan elimination, so that the LU solve of the coarsest grid for
//    a block of right-hand sides becomes one dense matrix product.
#include "common.hpp"
#include "kernels.hpp"
#include "tile_gemm.hpp"

namespace helm {

__device__ inline cx<double> cdiv(cx<double> a, cx<double> b) {
  const double d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
__device__ inline cx<double> tocx(c128 v) { return {v.re, v.im}; }
__device__ inline c128 toc(cx<double> v) { return {v.re, v.im}; }

__global__ void k_fine_coef(int64_t N, const double* __restrict__ m, const double* __restrict__ gamma, double w2,
                            double beta, double wjac, double lap, c128* __restrict__ dH, c128* __restrict__ dM,
                            c128* __restrict__ dw) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double mw = w2 * m[i];
  const cx<double> h = {lap - mw, mw * gamma[i]};
  const cx<double> s = {lap - mw, mw * (gamma[i] + beta)};
  dH[i] = toc(h);
  dM[i] = toc(s);
  dw[i] = toc(cdiv(cx<double>{wjac, 0.0}, s));
}

void launch_fine_coef(int dim, int64_t N, const double* m, const double* gamma, double omega, double beta,
                      double wjac, const double ih[3], c128* dH, c128* dM, c128* dw, hipStream_t s) {
  double lap = 0.0;
  for (int a = 0; a < dim; ++a) lap += 2.0 * ih[a];
  hipLaunchKernelGGL(k_fine_coef, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, m, gamma, omega * omega,
                     beta, wjac, lap, dH, dM, dw);
}

// Fine coupling M[f1, f1+s] of the 5/7-point shifted operator.
struct FineOp {
  const c128* dM;
  double ih[3];
  __device__ cx<double> operator()(int64_t f1, int sx, int sy, int sz) const {
    const int nz = (sx != 0) + (sy != 0) + (sz != 0);
    if (nz == 0) return tocx(dM[f1]);
    if (nz > 1) return {0.0, 0.0};
    const double v = sx ? ih[0] : (sy ? ih[1] : ih[2]);
    return {-v, 0.0};
  }
};
// Coupling of a stored 3^d stencil.
template <int DIM> struct GalOp {
  const c128* st;
  __device__ cx<double> operator()(int64_t f1, int sx, int sy, int sz) const {
    const int o = (sx + 1) + 3 * (sy + 1) + (DIM == 3 ? 9 * (sz + 1) : 0);
    return tocx(st[f1 * (DIM == 3 ? 27 : 9) + o]);
  }
};

// stc[J][o] = 2^-d sum_{f1 ~ J} sum_{f2 ~ J+o} P[f1,J] M[f1,f2] P[f2,J+o]
template <int DIM, class OP>
__global__ void k_galerkin(Geo gf, Geo gc, OP op, c128* __restrict__ stc) {
  constexpr int NS = DIM == 3 ? 27 : 9;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= gc.npts * NS) return;
  const int64_t J = t / NS;
  const int o = (int)(t - J * NS);
  const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = DIM == 3 ? o / 9 - 1 : 0;
  int X, Y, Z;
  coords(gc, J, X, Y, Z);
  const int IX = X + ox, IY = Y + oy, IZ = Z + oz;
  cx<double> acc = {0.0, 0.0};
  if (IX >= 0 && IX < gc.nx && IY >= 0 && IY < gc.ny && IZ >= 0 && IZ < gc.nz) {
    const int zlo = DIM == 3 ? -1 : 0, zhi = DIM == 3 ? 1 : 0;
    for (int dz = zlo; dz <= zhi; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int f1x = 2 * X + 1 + dx, f1y = 2 * Y + 1 + dy, f1z = DIM == 3 ? 2 * Z + 1 + dz : 0;
          const double w1 = (dx ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * (dz ? 0.5 : 1.0);
          const int64_t f1 = ((int64_t)f1z * gf.ny + f1y) * gf.nx + f1x;
          for (int sz = zlo; sz <= zhi; ++sz)
            for (int sy = -1; sy <= 1; ++sy)
              for (int sx = -1; sx <= 1; ++sx) {
                const int f2x = f1x + sx, f2y = f1y + sy, f2z = f1z + sz;
                if (f2x < 0 || f2x >= gf.nx || f2y < 0 || f2y >= gf.ny || f2z < 0 || f2z >= gf.nz) continue;
                const int ex = f2x - (2 * IX + 1), ey = f2y - (2 * IY + 1), ez = DIM == 3 ? f2z - (2 * IZ + 1) : 0;
                if (ex < -1 || ex > 1 || ey < -1 || ey > 1 || ez < -1 || ez > 1) continue;
                const double w2 = (ex ? 0.5 : 1.0) * (ey ? 0.5 : 1.0) * (ez ? 0.5 : 1.0);
                const cx<double> a = op(f1, sx, sy, sz);
                acc = acc + (w1 * w2) * a;
              }
        }
    acc = (DIM == 3 ? 0.125 : 0.25) * acc;
  }
  stc[t] = toc(acc);
}

void launch_galerkin_from_fine(int dim, const Geo& gf, const Geo& gc, const c128* dM, const double ih[3], c128* stc,
                               hipStream_t s) {
  FineOp op;
  op.dM = dM;
  op.ih[0] = ih[0];
  op.ih[1] = ih[1];
  op.ih[2] = ih[2];
  const int NS = dim == 3 ? 27 : 9;
  const dim3 gr((unsigned)((gc.npts * NS + 255) / 256));
  if (dim == 3)
    hipLaunchKernelGGL((k_galerkin<3, FineOp>), gr, dim3(256), 0, s, gf, gc, op, stc);
  else
    hipLaunchKernelGGL((k_galerkin<2, FineOp>), gr, dim3(256), 0, s, gf, gc, op, stc);
}

void launch_galerkin_from_gal(int dim, const Geo& gf, const Geo& gc, const c128* stf, c128* stc, hipStream_t s) {
  const int NS = dim == 3 ? 27 : 9;
  const dim3 gr((unsigned)((gc.npts * NS + 255) / 256));
  if (dim == 3)
    hipLaunchKernelGGL((k_galerkin<3, GalOp<3>>), gr, dim3(256), 0, s, gf, gc, GalOp<3>{stf}, stc);
  else
    hipLaunchKernelGGL((k_galerkin<2, GalOp<2>>), gr, dim3(256), 0, s, gf, gc, GalOp<2>{stf}, stc);
}

__global__ void k_gal_dw(int64_t N, int NS, const c128* __restrict__ st, double wjac, c128* __restrict__ dw) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  dw[i] = toc(cdiv(cx<double>{wjac, 0.0}, tocx(st[i * NS + NS / 2])));
}

void launch_gal_dw(int dim, int64_t N, const c128* st, double wjac, c128* dw, hipStream_t s) {
  hipLaunchKernelGGL(k_gal_dw, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, dim == 3 ? 27 : 9, st, wjac, dw);
}

__global__ void k_assemble(Geo g, int NS, const c128* __restrict__ st, c128* __restrict__ A) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.npts * NS) return;
  const int64_t i = t / NS;
  const int o = (int)(t - i * NS);
  const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = NS == 27 ? o / 9 - 1 : 0;
  int x, y, z;
  coords(g, i, x, y, z);
  x += ox;
  y += oy;
  z += oz;
  if (x < 0 || x >= g.nx || y < 0 || y >= g.ny || z < 0 || z >= g.nz) return;
  const int64_t j = ((int64_t)z * g.ny + y) * g.nx + x;
  A[i * g.npts + j] = st[t];
}

void launch_assemble_dense(int dim, const Geo& g, const c128* st, c128* A, hipStream_t s) {
  const int NS = dim == 3 ? 27 : 9;
  hipMemsetAsync(A, 0, sizeof(c128) * g.npts * g.npts, s);
  hipLaunchKernelGGL(k_assemble, dim3((unsigned)((g.npts * NS + 255) / 256)), dim3(256), 0, s, g, NS, st, A);
}

__global__ void k_narrow(int64_t n, const c128* __restrict__ a, c64* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = c64{(float)a[i].re, (float)a[i].im};
}
void launch_narrow(int64_t n, const c128* a, c64* b, hipStream_t s) {
  hipLaunchKernelGGL(k_narrow, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, a, b);
}

// ---------------------------------------------------------------------------
// Complex GEMM, C = alpha A B + beta C, row-major: one 64x64 tile per
// 256-thread workgroup (gemm_tile).
// ---------------------------------------------------------------------------
template <class S, class T>
__global__ __launch_bounds__(256) void k_gemm(int64_t M, int64_t N, int64_t K, cx<T> alpha, const S* __restrict__ A,
                                              int64_t lda, const S* __restrict__ B, int64_t ldb, cx<T> beta,
                                              S* __restrict__ C, int64_t ldc) {
  __shared__ cx<T> As[GEMM_BK][GEMM_BM + 1];
  __shared__ cx<T> Bs[GEMM_BK][GEMM_BN + 1];
  gemm_tile<S, T>(blockIdx.x, blockIdx.y, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, As, Bs);
}

void launch_gemm(Prec p, int64_t M, int64_t N, int64_t K, c128 alpha, const void* A, int64_t lda, const void* B,
                 int64_t ldb, c128 beta, void* C, int64_t ldc, hipStream_t s) {
  const dim3 gr((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64));
  if (p == P64) {
    hipLaunchKernelGGL((k_gemm<c128, double>), gr, dim3(256), 0, s, M, N, K, cx<double>{alpha.re, alpha.im},
                       (const c128*)A, lda, (const c128*)B, ldb, cx<double>{beta.re, beta.im}, (c128*)C, ldc);
  } else if (p == P32) {
    hipLaunchKernelGGL((k_gemm<c64, float>), gr, dim3(256), 0, s, M, N, K,
                       cx<float>{(float)alpha.re, (float)alpha.im}, (const c64*)A, lda, (const c64*)B, ldb,
                       cx<float>{(float)beta.re, (float)beta.im}, (c64*)C, ldc);
  } else {
    fatal_combo("launch_gemm");
  }
}

// ---------------------------------------------------------------------------
// Blocked Gauss-Jordan inversion without pivoting.
// ---------------------------------------------------------------------------
// In-place inverse of a small nb x nb block held in LDS (one workgroup).
__global__ __launch_bounds__(256) void k_small_gj(int nb, c128* __restrict__ D, int* __restrict__ fail) {
  extern __shared__ cx<double> sm[];
  cx<double>* A = sm;            // nb x nb
  cx<double>* col = sm + nb * nb;  // nb
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) A[e] = tocx(D[e]);
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    const cx<double> piv = A[k * nb + k];
    if (piv.re == 0.0 && piv.im == 0.0) {
      if (threadIdx.x == 0) *fail = 1;
      return;
    }
    const cx<double> p = cdiv(cx<double>{1.0, 0.0}, piv);
    __syncthreads();
    for (int j = threadIdx.x; j < nb; j += blockDim.x) {
      const cx<double> v = j == k ? cx<double>{1.0, 0.0} : A[k * nb + j];
      A[k * nb + j] = p * v;
    }
    for (int i = threadIdx.x; i < nb; i += blockDim.x) col[i] = A[i * nb + k];
    __syncthreads();
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
      const int i = e / nb, j = e % nb;
      if (i == k) continue;
      const cx<double> base = j == k ? cx<double>{0.0, 0.0} : A[e];
      A[e] = base - col[i] * A[k * nb + j];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) D[e] = toc(A[e]);
}

// Copy a rectangular sub-matrix (rows r0.., cols c0..) of a row-major matrix.
__global__ void k_copy_sub(int64_t rows, int64_t cols, const c128* __restrict__ src, int64_t lds,
                           c128* __restrict__ dst, int64_t ldd) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * cols) return;
  const int64_t r = t / cols, c = t - r * cols;
  dst[r * ldd + c] = src[r * lds + c];
}
__global__ void k_zero_rows(int64_t r0, int64_t nr, int64_t cols, c128* __restrict__ A, int64_t lda) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nr * cols) return;
  const int64_t r = t / cols, c = t - r * cols;
  A[(r0 + r) * lda + c] = c128{0.0, 0.0};
}

static inline dim3 g1(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

int gauss_jordan_inverse(int64_t n, c128* A, int nb, c128* work, hipStream_t s) {
  c128* Pc = work;            // n x nb
  c128* Rw = work + n * nb;   // nb x n
  c128* D = Rw + n * nb;      // nb x nb
  int* dfail = reinterpret_cast<int*>(D + (int64_t)nb * nb);
  hipMemsetAsync(dfail, 0, sizeof(int), s);
  const c128 one{1.0, 0.0}, zero{0.0, 0.0}, mone{-1.0, 0.0};
  for (int64_t k = 0; k < n; k += nb) {
    const int b = (int)((n - k) < nb ? (n - k) : nb);
    // D = A[K,K]; D <- D^-1
    hipLaunchKernelGGL(k_copy_sub, g1((int64_t)b * b), dim3(256), 0, s, (int64_t)b, (int64_t)b, A + k * n + k, n, D,
                       (int64_t)b);
    hipLaunchKernelGGL(k_small_gj, dim3(1), dim3(256), (size_t)(b * b + b) * sizeof(cx<double>), s, b, D, dfail);
    // Pc = A[:, K] with rows K zeroed
    hipLaunchKernelGGL(k_copy_sub, g1(n * b), dim3(256), 0, s, n, (int64_t)b, A + k, n, Pc, (int64_t)b);
    hipLaunchKernelGGL(k_zero_rows, g1((int64_t)b * b), dim3(256), 0, s, k, (int64_t)b, (int64_t)b, Pc, (int64_t)b);
    // Rw = D^-1 A[K, :]
    launch_gemm(P64, b, n, b, one, D, b, A + k * n, n, zero, Rw, n, s);
    // A -= Pc Rw   (rows K untouched since Pc rows K are zero)
    launch_gemm(P64, n, n, b, mone, Pc, b, Rw, n, one, A, n, s);
    // A[K, :] = Rw
    hipLaunchKernelGGL(k_copy_sub, g1((int64_t)b * n), dim3(256), 0, s, (int64_t)b, n, Rw, n, A + k * n, n);
    // A[:, K] = -Pc D^-1 ; then A[K,K] = D^-1
    launch_gemm(P64, n, b, b, mone, Pc, b, D, b, zero, A + k, n, s);
    hipLaunchKernelGGL(k_copy_sub, g1((int64_t)b * b), dim3(256), 0, s, (int64_t)b, (int64_t)b, D, (int64_t)b,
                       A + k * n + k, n);
  }
  int hfail = 0;
  if (hipMemcpyAsync(&hfail, dfail, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return -1;
  if (hipStreamSynchronize(s) != hipSuccess) return -1;
  return hfail ? 1 : 0;
}

}  // namespace helm
