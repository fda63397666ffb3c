// k_krylov.hip -- FP64 kernels of block FGMRES (section 5.3, "block FGMRES(5)").
//
// A block of P right-hand sides is split into groups of pb columns; each
// group is an independent block-Krylov solve and all groups share every
// launch. Vectors are point-major c128 blocks [N][ld].
//
//  - block Gram products V_i^H W: lanes own one column, loop over a grid
//    stride of points, reduce across lanes through LDS, then a second pass
//    sums the per-workgroup partials in a fixed order (deterministic);
//  - block updates W -= sum_i V_i H_i, V = W R^-1 and X += sum_j Z_j Y_j:
//    lanes own one (point, column) entry; the pb values of the group at
//    that point are read once per lane group (broadcast through L1);
//  - Cholesky of the pb x pb Gram matrix (CholQR) and the small block
//    least-squares problem (Householder) run in one workgroup per group.
#include "common.hpp"
#include "kernels.hpp"

namespace helm {

__device__ inline cx<double> tcx(c128 v) { return {v.re, v.im}; }
__device__ inline c128 fcx(cx<double> v) { return {v.re, v.im}; }

constexpr int GRAM_MAXACC = 16;
constexpr int GRAM_BLOCKS = 2048;

// part[blk][i][c][a] for i < k, c < P, a < na (a offset by a0 in the group).
// KN = k * na accumulators, a compile-time count so that every load of a
// point is issued before its multiply-adds (many loads in flight per wave).
template <class S, int KN>
__global__ __launch_bounds__(256) void k_gram_part(int64_t N, int ld, int P, int pb, int k, int a0, int na,
                                                   PtrList X, const S* __restrict__ Y,
                                                   c128* __restrict__ part) {
  extern __shared__ cx<double> red[];  // [256][KN]
  const int tid = threadIdx.x;
  const int PT = 256 / P;
  const int c = tid % P, r = tid / P;
  cx<double> acc[KN];
#pragma unroll
  for (int e = 0; e < KN; ++e) acc[e] = {0.0, 0.0};
  const int64_t chunk = (N + gridDim.x - 1) / gridDim.x;
  const int64_t nb0 = (int64_t)blockIdx.x * chunk;
  const int64_t nb1 = nb0 + chunk < N ? nb0 + chunk : N;
  if (r < PT) {
    const int cb = (c / pb) * pb + a0;
    const S* xp[KN];
#pragma unroll
    for (int e = 0; e < KN; ++e) {
      const int i = e / na, a = e - i * na;
      xp[e] = static_cast<const S*>(X.p[i]) + cb + a;
    }
    for (int64_t n = nb0 + r; n < nb1; n += PT) {
      const S yv = Y[n * ld + c];
      S xv[KN];
#pragma unroll
      for (int e = 0; e < KN; ++e) xv[e] = xp[e][n * ld];
      const cx<double> y = {(double)yv.re, (double)yv.im};
#pragma unroll
      for (int e = 0; e < KN; ++e) cfmac(acc[e], cx<double>{(double)xv[e].re, (double)xv[e].im}, y);
    }
  }
#pragma unroll
  for (int e = 0; e < KN; ++e) red[tid * KN + e] = acc[e];
  __syncthreads();
  for (int o = tid; o < P * KN; o += 256) {
    const int cc = o / KN, e = o - cc * KN;
    cx<double> s = {0.0, 0.0};
    for (int rr = 0; rr < PT; ++rr) s = s + red[(rr * P + cc) * KN + e];
    const int i = e / na, a = e - i * na;
    part[((((int64_t)i * P + cc) * na + a)) * gridDim.x + blockIdx.x] = fcx(s);
  }
}

template <class S, int KN>
static void gram_part_launch(int nblk, hipStream_t s, int64_t N, int ld, int P, int pb, int k, int a0, int na,
                             const PtrList& X, const void* Y, c128* part) {
  const size_t shm = sizeof(cx<double>) * 256 * KN;
  hipLaunchKernelGGL((k_gram_part<S, KN>), dim3(nblk), dim3(256), shm, s, N, ld, P, pb, k, a0, na, X,
                     (const S*)Y, part);
}

template <class S>
static void gram_part_dispatch(int kn, int nblk, hipStream_t s, int64_t N, int ld, int P, int pb, int k, int a0,
                               int na, const PtrList& X, const void* Y, c128* part) {
  switch (kn) {
#define HELM_KN(v) \
  case v: gram_part_launch<S, v>(nblk, s, N, ld, P, pb, k, a0, na, X, Y, part); break;
    HELM_KN(1) HELM_KN(2) HELM_KN(3) HELM_KN(4) HELM_KN(5) HELM_KN(6) HELM_KN(7) HELM_KN(8)
    HELM_KN(9) HELM_KN(10) HELM_KN(11) HELM_KN(12) HELM_KN(13) HELM_KN(14) HELM_KN(15) HELM_KN(16)
#undef HELM_KN
    default: fatal_combo("gram_part_dispatch");
  }
}

// G[i][c][a0+a] = sum over blocks of part[o][blk], one workgroup per output:
// each lane sums a fixed interleaved subset, then a fixed-order tree in LDS
// (deterministic).
__global__ __launch_bounds__(256) void k_gram_final(int nblk, int P, int pb, int k, int i0, int a0, int na,
                                                    const c128* __restrict__ part, c128* __restrict__ G) {
  __shared__ cx<double> red[256];
  const int o = blockIdx.x;
  const c128* p = part + (int64_t)o * nblk;
  cx<double> s = {0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += 256) s = s + tcx(p[b]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int a = o % na, c = (o / na) % P, i = o / (na * P);
    G[((int64_t)(i0 + i) * P + c) * pb + a0 + a] = fcx(red[0]);
  }
}

int64_t gram_part_elems(int P) { return (int64_t)GRAM_BLOCKS * GRAM_MAXACC * P; }

// Workgroups for a column reduction over N points: at least 8 loop trips
// per lane (PT = 256/P points per trip), at most GRAM_BLOCKS, so that small
// grids (the 47^3 coarsest level) still fill the device.
static int part_blocks(int64_t N, int P) {
  const int64_t pts = (int64_t)(256 / P) * 8;
  int64_t nb = (N + pts - 1) / pts;
  if (nb > GRAM_BLOCKS) nb = GRAM_BLOCKS;
  return nb < 1 ? 1 : (int)nb;
}

void launch_gram(Prec p, int64_t N, int ld, int P, int pb, int k, const PtrList& X, const void* Y, c128* part,
                 c128* G, hipStream_t s) {
  if (p != P64 && p != P32) fatal_combo("launch_gram");
  if (P > 256 || P % pb != 0) fatal_combo("launch_gram");
  const int nblk = part_blocks(N, P);
  const int na = pb < GRAM_MAXACC ? pb : GRAM_MAXACC;
  const int kk = GRAM_MAXACC / na;
  for (int i0 = 0; i0 < k; i0 += kk) {
    const int kc = (k - i0) < kk ? (k - i0) : kk;
    for (int a0 = 0; a0 < pb; a0 += na) {
      PtrList sub{};
      for (int i = 0; i < kc; ++i) sub.p[i] = X.p[i0 + i];
      if (p == P64)
        gram_part_dispatch<c128>(kc * na, nblk, s, N, ld, P, pb, kc, a0, na, sub, Y, part);
      else
        gram_part_dispatch<c64>(kc * na, nblk, s, N, ld, P, pb, kc, a0, na, sub, Y, part);
      const int outs = kc * P * na;
      hipLaunchKernelGGL(k_gram_final, dim3(outs), dim3(256), 0, s, nblk, P, pb, kc, i0, a0, na, part, G);
    }
  }
}

// ---------------------------------------------------------------------------
template <class SX, class SY>
__global__ __launch_bounds__(256) void k_block_update(int mode, int64_t N, int ld, int P, int pb, int k,
                                                      PtrList X, const c128* __restrict__ C,
                                                      SY* __restrict__ Y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * P) return;
  const int64_t n = t / P;
  const int c = (int)(t - n * P);
  const int cb = (c / pb) * pb;
  cx<double> acc = {0.0, 0.0};
  for (int i = 0; i < k; ++i) {
    const SX* xi = static_cast<const SX*>(X.p[i]) + n * ld + cb;
    const c128* ci = C + ((int64_t)i * P + c) * pb;
    for (int a = 0; a < pb; ++a) {
      const SX xv = xi[a];
      cfma(acc, cx<double>{(double)xv.re, (double)xv.im}, tcx(ci[a]));
    }
  }
  SY* yp = Y + n * ld + c;
  cx<double> r = acc;
  if (mode != 1) {
    const SY yv = *yp;
    const cx<double> y = {(double)yv.re, (double)yv.im};
    r = mode == 0 ? y - acc : y + acc;
  }
  using E = decltype(yp->re);
  *yp = SY{(E)r.re, (E)r.im};
}

// Block size 1 with a compile-time vector count (loads issued together).
template <class SX, class SY, int KX>
__global__ __launch_bounds__(256) void k_update1(int mode, int64_t N, int ld, int P, PtrList X,
                                                 const c128* __restrict__ C, SY* __restrict__ Y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * P) return;
  const int64_t n = t / P;
  const int c = (int)(t - n * P);
  SX xv[KX];
#pragma unroll
  for (int i = 0; i < KX; ++i) xv[i] = static_cast<const SX*>(X.p[i])[n * ld + c];
  cx<double> acc = {0.0, 0.0};
#pragma unroll
  for (int i = 0; i < KX; ++i) cfma(acc, cx<double>{(double)xv[i].re, (double)xv[i].im}, tcx(C[(int64_t)i * P + c]));
  SY* yp = Y + n * ld + c;
  cx<double> r = acc;
  if (mode != 1) {
    const SY yv = *yp;
    const cx<double> y = {(double)yv.re, (double)yv.im};
    r = mode == 0 ? y - acc : y + acc;
  }
  using E = decltype(yp->re);
  *yp = SY{(E)r.re, (E)r.im};
}

template <class SX, class SY>
static void update1_dispatch(int kx, dim3 gr, hipStream_t s, int mode, int64_t N, int ld, int P, const PtrList& X,
                             const c128* C, void* Y) {
  switch (kx) {
#define HELM_KX(v)                                                                                              \
  case v:                                                                                                       \
    hipLaunchKernelGGL((k_update1<SX, SY, v>), gr, dim3(256), 0, s, mode, N, ld, P, X, C, (SY*)Y);          \
    break;
    HELM_KX(1) HELM_KX(2) HELM_KX(3) HELM_KX(4) HELM_KX(5) HELM_KX(6) HELM_KX(7) HELM_KX(8)
    HELM_KX(9) HELM_KX(10) HELM_KX(11) HELM_KX(12) HELM_KX(13) HELM_KX(14) HELM_KX(15) HELM_KX(16)
#undef HELM_KX
    default: fatal_combo("update1_dispatch");
  }
}

void launch_block_update(int mode, Prec px, Prec py, int64_t N, int ld, int P, int pb, int k, const PtrList& X,
                         const c128* C, void* Y, hipStream_t s) {
  const dim3 gr((unsigned)((N * P + 255) / 256));
  if (k > MAXPTR) fatal_combo("launch_block_update");
  if (pb == 1) {
    // chunks of at most 16 vectors; later chunks accumulate into Y
    for (int i0 = 0; i0 < k; i0 += 16) {
      const int kx = (k - i0) < 16 ? (k - i0) : 16;
      PtrList sub{};
      for (int i = 0; i < kx; ++i) sub.p[i] = X.p[i0 + i];
      const int md = (i0 == 0) ? mode : (mode == 1 ? 2 : mode);
      const c128* Cs = C + (int64_t)i0 * P;
      if (px == P64 && py == P64)
        update1_dispatch<c128, c128>(kx, gr, s, md, N, ld, P, sub, Cs, Y);
      else if (px == P32 && py == P64)
        update1_dispatch<c64, c128>(kx, gr, s, md, N, ld, P, sub, Cs, Y);
      else if (px == P32 && py == P32)
        update1_dispatch<c64, c64>(kx, gr, s, md, N, ld, P, sub, Cs, Y);
      else
        fatal_combo("launch_block_update");
    }
    return;
  }
  if (px == P64 && py == P64)
    hipLaunchKernelGGL((k_block_update<c128, c128>), gr, dim3(256), 0, s, mode, N, ld, P, pb, k, X, C, (c128*)Y);
  else if (px == P32 && py == P64)
    hipLaunchKernelGGL((k_block_update<c64, c128>), gr, dim3(256), 0, s, mode, N, ld, P, pb, k, X, C, (c128*)Y);
  else if (px == P32 && py == P32)
    hipLaunchKernelGGL((k_block_update<c64, c64>), gr, dim3(256), 0, s, mode, N, ld, P, pb, k, X, C, (c64*)Y);
  else
    fatal_combo("launch_block_update");
}

// ---------------------------------------------------------------------------
// Cholesky G = R^H R per group (one workgroup each), R upper, and R^-1, with
// deflation of dependent columns. Column j's reduced diagonal d_j (the
// squared norm of its part independent of the columns before it) is
// compared with rtol times its own squared norm G_jj and with tol times the
// largest G_aa: at or below either, column j is dropped (row j of R and
// row and column j of R^-1 are zero, so the basis gets a zero column and
// W = Q R holds for column j to within sqrt(d_j)). flag[g] = 1 when a
// column was dropped or a kept one has d_j < 1e-4 G_jj (the product
// W R^-1 then has lost orthogonality of order eps G_jj / d_j, and a second
// pass is advised), else 0.
// G layout: Gm[a][b] = G[(g*pb + b)*pb + a]. Outputs: R[g][a][b] row-major,
// RinvC in update layout: RinvC[(g*pb + b)*pb + a] = Rinv[a][b].
// ---------------------------------------------------------------------------
// The working matrices are static LDS sized for the largest group (2 x 64 KB
// at 64 columns; gfx950 gives a workgroup up to 160 KB).
constexpr int CHOL_MAXPB = 64;
__global__ __launch_bounds__(256) void k_cholqr_small(int pb, const c128* __restrict__ G, c128* __restrict__ R,
                                                      c128* __restrict__ RinvC, int* __restrict__ flag, double tol,
                                                      double rtol) {
  __shared__ cx<double> A[CHOL_MAXPB * CHOL_MAXPB];   // pb x pb working copy (upper part becomes R)
  __shared__ cx<double> Ri[CHOL_MAXPB * CHOL_MAXPB];  // pb x pb inverse
  __shared__ double dmax;
  __shared__ double gd[CHOL_MAXPB];
  __shared__ int drp[CHOL_MAXPB];
  __shared__ int ill;
  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  for (int e = tid; e < pb * pb; e += blockDim.x) {
    const int a = e / pb, b = e % pb;
    A[e] = tcx(G[((int64_t)g * pb + b) * pb + a]);
  }
  if (tid == 0) {
    ill = 0;
    dmax = 0.0;
  }
  __syncthreads();
  if (tid == 0)
    for (int a = 0; a < pb; ++a) {
      gd[a] = A[a * pb + a].re;
      dmax = fmax(dmax, gd[a]);
    }
  __syncthreads();
  for (int j = 0; j < pb; ++j) {
    // A[j][j] <- sqrt(A[j][j]) (already reduced by previous rows), or drop
    if (tid == 0) {
      const double d = A[j * pb + j].re;
      const int dr = !(d > tol * dmax) || !(d > rtol * gd[j]);
      drp[j] = dr;
      if (dr || d < 1e-4 * gd[j]) ill = 1;
      A[j * pb + j] = {dr ? 0.0 : sqrt(d), 0.0};
    }
    __syncthreads();
    if (drp[j]) {
      for (int b = j + 1 + tid; b < pb; b += blockDim.x) A[j * pb + b] = {0.0, 0.0};
      __syncthreads();
      continue;  // a zero row of R changes no later column
    }
    const double inv = 1.0 / A[j * pb + j].re;
    for (int b = j + 1 + tid; b < pb; b += blockDim.x) A[j * pb + b] = inv * A[j * pb + b];
    __syncthreads();
    // trailing update A[a][b] -= conj(R[j][a]) R[j][b] for j < a <= b
    for (int e = tid; e < pb * pb; e += blockDim.x) {
      const int a = e / pb, b = e % pb;
      if (a > j && b >= a) {
        const cx<double> ra = A[j * pb + a], rb = A[j * pb + b];
        cfmac(A[e], cx<double>{-ra.re, -ra.im}, rb);
      }
    }
    __syncthreads();
  }
  if (tid == 0) flag[g] = ill;
  // Ri = R^-1 on the kept columns by back substitution, one column per lane;
  // rows and columns of dropped columns are zero (a dropped l contributes
  // nothing to the sums below because Ri[l][b] = 0)
  for (int b = tid; b < pb; b += blockDim.x) {
    for (int a = pb - 1; a >= 0; --a) {
      if (a > b || drp[a] || drp[b]) {
        Ri[a * pb + b] = {0.0, 0.0};
        continue;
      }
      cx<double> s = {a == b ? 1.0 : 0.0, 0.0};
      for (int l = a + 1; l <= b; ++l) s = s - A[a * pb + l] * Ri[l * pb + b];
      Ri[a * pb + b] = (1.0 / A[a * pb + a].re) * s;
    }
  }
  __syncthreads();
  for (int e = tid; e < pb * pb; e += blockDim.x) {
    const int a = e / pb, b = e % pb;
    R[(int64_t)g * pb * pb + e] = a <= b ? fcx(A[e]) : c128{0.0, 0.0};
    RinvC[((int64_t)g * pb + b) * pb + a] = fcx(Ri[e]);
  }
}

void launch_cholqr_small(int ng, int pb, const c128* G, c128* R, c128* Rinv, int* flag, double tol, double rtol,
                         hipStream_t s) {
  if (pb < 1 || pb > CHOL_MAXPB) fatal_combo("launch_cholqr_small");
  hipLaunchKernelGGL(k_cholqr_small, dim3(ng), dim3(256), 0, s, pb, G, R, Rinv, flag, tol, rtol);
}

// R <- R2 R per group (both upper triangular, row-major [g][a][b]): the
// factor of a block after a second CholQR pass (W = Q1 R, Q1 = Q2 R2).
__global__ __launch_bounds__(256) void k_rmul_small(int pb, const c128* __restrict__ R2, c128* __restrict__ R) {
  __shared__ cx<double> A[CHOL_MAXPB * CHOL_MAXPB];
  __shared__ cx<double> B[CHOL_MAXPB * CHOL_MAXPB];
  const int64_t o = (int64_t)blockIdx.x * pb * pb;
  for (int e = threadIdx.x; e < pb * pb; e += blockDim.x) {
    A[e] = tcx(R2[o + e]);
    B[e] = tcx(R[o + e]);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < pb * pb; e += blockDim.x) {
    const int a = e / pb, b = e % pb;
    cx<double> acc = {0.0, 0.0};
    for (int l = a; l <= b; ++l) cfmac(acc, A[a * pb + l], B[l * pb + b]);
    R[o + e] = fcx(acc);
  }
}

void launch_rmul_small(int ng, int pb, const c128* R2, c128* R, hipStream_t s) {
  if (pb < 1 || pb > CHOL_MAXPB) fatal_combo("launch_rmul_small");
  hipLaunchKernelGGL(k_rmul_small, dim3(ng), dim3(256), 0, s, pb, R2, R);
}

// ---------------------------------------------------------------------------
// Block least squares per group: min ||[S; 0] - Hbar Y||_F by Householder.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_block_ls(int pb, int j, int P, const c128* __restrict__ Hb, int ldh,
                                                  int64_t hstride, const c128* __restrict__ S, c128* __restrict__ Yc,
                                                  double* __restrict__ est, c128* __restrict__ scratch,
                                                  const int* __restrict__ active) {
  const int g = blockIdx.x, tid = threadIdx.x;
  const int r = (j + 2) * pb, cc = (j + 1) * pb;
  const int ncol = cc + pb;
  cx<double>* M = reinterpret_cast<cx<double>*>(scratch) + (int64_t)g * r * ncol;  // col-major r x ncol
  __shared__ double sred[256];
  __shared__ cx<double> salpha;
  __shared__ double svn2;
  __shared__ int skip;
  if (active && !active[g]) {
    for (int e = tid; e < (j + 1) * pb * pb; e += blockDim.x) {
      const int jj = e / (pb * pb), rem = e % (pb * pb), b = rem / pb, a = rem % pb;
      Yc[((int64_t)jj * P + g * pb + b) * pb + a] = c128{0.0, 0.0};
    }
    for (int b = tid; b < pb; b += blockDim.x) est[g * pb + b] = 0.0;
    return;
  }
  const c128* H = Hb + (int64_t)g * hstride;
  for (int e = tid; e < r * cc; e += blockDim.x) {
    const int col = e / r, row = e % r;
    M[e] = tcx(H[(int64_t)col * ldh + row]);
  }
  for (int e = tid; e < r * pb; e += blockDim.x) {
    const int b = e / r, row = e % r;
    M[(int64_t)(cc + b) * r + row] = row < pb ? tcx(S[((int64_t)g * pb + row) * pb + b]) : cx<double>{0.0, 0.0};
  }
  __syncthreads();
  for (int q = 0; q < cc; ++q) {
    double part = 0.0;
    for (int i = q + tid; i < r; i += blockDim.x) {
      const cx<double> v = M[(int64_t)q * r + i];
      part += v.re * v.re + v.im * v.im;
    }
    sred[tid] = part;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) sred[tid] += sred[tid + w];
      __syncthreads();
    }
    if (tid == 0) {
      const double nrm = sqrt(sred[0]);
      const cx<double> x0 = M[(int64_t)q * r + q];
      const double ax = sqrt(x0.re * x0.re + x0.im * x0.im);
      skip = nrm == 0.0;
      const cx<double> ph = ax > 0.0 ? cx<double>{x0.re / ax, x0.im / ax} : cx<double>{1.0, 0.0};
      salpha = {-ph.re * nrm, -ph.im * nrm};
      const cx<double> v0 = x0 - salpha;
      svn2 = sred[0] - ax * ax + (v0.re * v0.re + v0.im * v0.im);
      M[(int64_t)q * r + q] = v0;  // reflector v stored in column q (rows q..r-1)
    }
    __syncthreads();
    if (!skip) {
      const double f = 2.0 / svn2;
      for (int col = q + 1 + tid; col < ncol; col += blockDim.x) {
        cx<double> d = {0.0, 0.0};
        for (int i = q; i < r; ++i) cfmac(d, M[(int64_t)q * r + i], M[(int64_t)col * r + i]);
        d = f * d;
        for (int i = q; i < r; ++i) {
          const cx<double> v = M[(int64_t)q * r + i];
          M[(int64_t)col * r + i] = M[(int64_t)col * r + i] - v * d;
        }
      }
    }
    __syncthreads();
    if (tid == 0) M[(int64_t)q * r + q] = salpha;  // diagonal of R
    __syncthreads();
  }
  // back substitution per right-hand-side column; R = upper part of M[:, :cc]
  for (int b = tid; b < pb; b += blockDim.x) {
    cx<double>* rhs = M + (int64_t)(cc + b) * r;
    double e2 = 0.0;
    for (int i = cc; i < r; ++i) e2 += rhs[i].re * rhs[i].re + rhs[i].im * rhs[i].im;
    est[g * pb + b] = sqrt(e2);
    for (int i = cc - 1; i >= 0; --i) {
      cx<double> s = rhs[i];
      for (int l = i + 1; l < cc; ++l) s = s - M[(int64_t)l * r + i] * rhs[l];
      const cx<double> d = M[(int64_t)i * r + i];
      const double dd = d.re * d.re + d.im * d.im;
      rhs[i] = dd > 0.0 ? cx<double>{(s.re * d.re + s.im * d.im) / dd, (s.im * d.re - s.re * d.im) / dd}
                        : cx<double>{0.0, 0.0};
    }
    for (int i = 0; i < cc; ++i) {
      const int jj = i / pb, a = i % pb;
      Yc[((int64_t)jj * P + g * pb + b) * pb + a] = fcx(rhs[i]);
    }
  }
}

void launch_block_ls(int ng, int pb, int j, const c128* Hb, int ldh, int64_t hstride, const c128* S, c128* Y,
                     int64_t ystride, double* est, c128* scratch, const int* active, hipStream_t s) {
  (void)ystride;
  hipLaunchKernelGGL(k_block_ls, dim3(ng), dim3(256), 0, s, pb, j, ng * pb, Hb, ldh, hstride, S, Y, est, scratch,
                     active);
}

// ---------------------------------------------------------------------------
__global__ void k_diag_real(int P, const c128* __restrict__ G, double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < P) out[c] = G[c].re;
}

void launch_diag_real(int P, const c128* G, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_real, dim3((P + 255) / 256), dim3(256), 0, s, P, G, out);
}

void launch_colnorm2(Prec p, int64_t N, int ld, int P, const void* X, c128* part, c128* G, double* out,
                     hipStream_t s) {
  PtrList xl{};
  xl.p[0] = X;
  launch_gram(p, N, ld, P, 1, 1, xl, X, part, G, s);
  hipLaunchKernelGGL(k_diag_real, dim3((P + 255) / 256), dim3(256), 0, s, P, G, out);
}

__global__ void k_mask_cols(int64_t N, int ld, int P, int pb, const int* __restrict__ active, c128* __restrict__ Y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * P) return;
  const int64_t n = t / P;
  const int c = (int)(t - n * P);
  if (!active[c / pb]) Y[n * ld + c] = c128{0.0, 0.0};
}
void launch_mask_cols(int64_t N, int ld, int P, int pb, const int* active, c128* Y, hipStream_t s) {
  hipLaunchKernelGGL(k_mask_cols, dim3((unsigned)((N * P + 255) / 256)), dim3(256), 0, s, N, ld, P, pb, active, Y);
}

template <class S>
__global__ void k_scale_cols(int64_t N, int ld, int P, const double* __restrict__ sc, const S* __restrict__ X,
                             S* __restrict__ Y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * P) return;
  const int64_t n = t / P;
  const int c = (int)(t - n * P);
  const S v = X[n * ld + c];
  using E = decltype(v.re);
  Y[n * ld + c] = S{(E)(sc[c] * v.re), (E)(sc[c] * v.im)};
}
void launch_scale_cols(Prec p, int64_t N, int ld, int P, const double* sc, const void* X, void* Y, hipStream_t s) {
  const dim3 gr((unsigned)((N * P + 255) / 256));
  if (p == P64)
    hipLaunchKernelGGL((k_scale_cols<c128>), gr, dim3(256), 0, s, N, ld, P, sc, (const c128*)X, (c128*)Y);
  else if (p == P32)
    hipLaunchKernelGGL((k_scale_cols<c64>), gr, dim3(256), 0, s, N, ld, P, sc, (const c64*)X, (c64*)Y);
  else
    fatal_combo("launch_scale_cols");
}

// ---------------------------------------------------------------------------
// Block size 1: Y[n][c] -= sum_i X_i[n][c] C[i][c], and the new ||Y_c||^2 as
// per-workgroup partials (same lane layout as the Gram kernel, so the final
// reduction is k_gram_final with k = na = pb = 1).
// ---------------------------------------------------------------------------
template <class S, int KX>
__global__ __launch_bounds__(256) void k_update_norm_part(int64_t N, int ld, int P, int with_norm, PtrList X,
                                                          const c128* __restrict__ C, S* __restrict__ Y,
                                                          c128* __restrict__ part, const double* __restrict__ osc) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int PT = 256 / P;
  const int c = tid % P, r = tid / P;
  const int64_t chunk = (N + gridDim.x - 1) / gridDim.x;
  const int64_t nb0 = (int64_t)blockIdx.x * chunk;
  const int64_t nb1 = nb0 + chunk < N ? nb0 + chunk : N;
  double nrm = 0.0;
  using E = decltype(Y->re);
  if (r < PT) {
    cx<double> coef[KX];
    const S* xp[KX];
#pragma unroll
    for (int i = 0; i < KX; ++i) {
      coef[i] = tcx(C[(int64_t)i * P + c]);
      xp[i] = static_cast<const S*>(X.p[i]) + c;
    }
    const double sc = osc ? osc[c] : 1.0;
    for (int64_t n = nb0 + r; n < nb1; n += PT) {
      const int64_t e = n * ld + c;
      const S yv = Y[e];
      S xv[KX];
#pragma unroll
      for (int i = 0; i < KX; ++i) xv[i] = xp[i][n * ld];
      cx<double> y = {(double)yv.re, (double)yv.im};
#pragma unroll
      for (int i = 0; i < KX; ++i) cfma(y, cx<double>{-(double)xv[i].re, -(double)xv[i].im}, coef[i]);
      if (osc) y = sc * y;
      const S out = S{(E)y.re, (E)y.im};
      Y[e] = out;
      nrm += (double)out.re * (double)out.re + (double)out.im * (double)out.im;
    }
  }
  if (!with_norm) return;
  red[tid] = nrm;
  __syncthreads();
  for (int cc = tid; cc < P; cc += 256) {
    double s = 0.0;
    for (int rr = 0; rr < PT; ++rr) s += red[rr * P + cc];
    part[(int64_t)cc * gridDim.x + blockIdx.x] = c128{s, 0.0};
  }
}

template <class S>
static void update_norm_dispatch(int kx, int nblk, hipStream_t s, int64_t N, int ld, int P, int with_norm,
                                 const PtrList& X, const c128* C, void* Y, c128* part, const double* osc) {
  switch (kx) {
#define HELM_KX(v)                                                                                             \
  case v:                                                                                                      \
    hipLaunchKernelGGL((k_update_norm_part<S, v>), dim3(nblk), dim3(256), 0, s, N, ld, P, with_norm, X, C, \
                       (S*)Y, part, osc);                                                                      \
    break;
    HELM_KX(1) HELM_KX(2) HELM_KX(3) HELM_KX(4) HELM_KX(5) HELM_KX(6) HELM_KX(7) HELM_KX(8)
    HELM_KX(9) HELM_KX(10) HELM_KX(11) HELM_KX(12) HELM_KX(13) HELM_KX(14) HELM_KX(15) HELM_KX(16)
#undef HELM_KX
    default: fatal_combo("update_norm_dispatch");
  }
}

void launch_update_norm(Prec p, int64_t N, int ld, int P, int k, const PtrList& X, const c128* C, void* Y,
                        c128* part, c128* G, double* nrm2, hipStream_t s, const double* osc) {
  if (P > 256 || k > MAXPTR) fatal_combo("launch_update_norm");
  const int nblk = part_blocks(N, P);
  // at most 16 vectors per pass; the norm comes from the last pass
  for (int i0 = 0; i0 < k; i0 += 16) {
    const int kx = (k - i0) < 16 ? (k - i0) : 16;
    PtrList sub{};
    for (int i = 0; i < kx; ++i) sub.p[i] = X.p[i0 + i];
    const int last = i0 + 16 >= k;
    // the output scale applies once, in the last pass
    const double* sc = last ? osc : nullptr;
    if (p == P64)
      update_norm_dispatch<c128>(kx, nblk, s, N, ld, P, last, sub, C + (int64_t)i0 * P, Y, part, sc);
    else if (p == P32)
      update_norm_dispatch<c64>(kx, nblk, s, N, ld, P, last, sub, C + (int64_t)i0 * P, Y, part, sc);
    else
      fatal_combo("launch_update_norm");
  }
  hipLaunchKernelGGL(k_gram_final, dim3(P), dim3(256), 0, s, nblk, P, 1, 1, 0, 0, 1, part, G);
  hipLaunchKernelGGL(k_diag_real, dim3((P + 255) / 256), dim3(256), 0, s, P, G, nrm2);
}

// From ||w||^2 per column (block size 1): R = ||w||, Rinv = 1/||w|| (0 and a
// breakdown flag when the column vanished, or is tiny against ref2).
__global__ void k_norm_to_r(int P, const double* __restrict__ n2, const double* __restrict__ ref2, double tol,
                            c128* __restrict__ R, c128* __restrict__ Rinv, int* __restrict__ flag) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P) return;
  const double v = n2[c];
  const bool bad = !(v > tol * (ref2 ? ref2[c] : 0.0)) || !(v > 0.0);
  const double nr = bad ? 0.0 : sqrt(v);
  R[c] = c128{nr, 0.0};
  Rinv[c] = c128{bad ? 0.0 : 1.0 / nr, 0.0};
  flag[c] = bad ? 1 : 0;
}
void launch_norm_to_r(int P, const double* n2, const double* ref2, double tol, c128* R, c128* Rinv, int* flag,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_norm_to_r, dim3((P + 255) / 256), dim3(256), 0, s, P, n2, ref2, tol, R, Rinv, flag);
}

// ---------------------------------------------------------------------------
// Block size 1 with an unnormalised basis: the stored vector v~_i = nu_i v_i
// (nu_i = ||v~_i||), W~ = H M(v~_j) = nu_j H z_j. From the raw Gram values
// g_i = v~_i^H W~ (i <= j): update coefficients c_i = g_i / nu_i^2 (so that
// W~ - sum c_i v~_i = nu_j (w - sum v_i h_ij)) and the Hessenberg entries
// h_ij = g_i / (nu_i nu_j), written to column j of Hbar (ld ldh per column).
// ---------------------------------------------------------------------------
__global__ void k_lazy_coef(int P, int j, const c128* __restrict__ Graw, const double* __restrict__ nu,
                            c128* __restrict__ C, c128* __restrict__ Hb, int ldh, int64_t hstride, int accumulate) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P) return;
  const double nj = nu[(int64_t)j * P + c];
  c128* H = Hb + (int64_t)c * hstride + (int64_t)j * ldh;
  for (int i = 0; i <= j; ++i) {
    const c128 g = Graw[(int64_t)i * P + c];
    const double ni = nu[(int64_t)i * P + c];
    const double a = ni > 0.0 ? 1.0 / (ni * ni) : 0.0;
    const double b = (ni > 0.0 && nj > 0.0) ? 1.0 / (ni * nj) : 0.0;
    C[(int64_t)i * P + c] = c128{g.re * a, g.im * a};
    const c128 h = accumulate ? H[i] : c128{0.0, 0.0};
    H[i] = c128{h.re + g.re * b, h.im + g.im * b};
  }
}
void launch_lazy_coef(int P, int j, const c128* Graw, const double* nu, c128* C, c128* Hb, int ldh, int64_t hstride,
                      int accumulate, hipStream_t s) {
  hipLaunchKernelGGL(k_lazy_coef, dim3((P + 63) / 64), dim3(64), 0, s, P, j, Graw, nu, C, Hb, ldh, hstride,
                     accumulate);
}
// nu_{j+1} = ||W~'||; h_{j+1,j} = nu_{j+1} / nu_j; breakdown flag when the new
// vector vanished against ||W~|| before orthogonalisation (ref2).
__global__ void k_lazy_next(int P, int j, const double* __restrict__ n2, const double* __restrict__ ref2, double tol,
                            double* __restrict__ nu, c128* __restrict__ Hb, int ldh, int64_t hstride,
                            int* __restrict__ flag) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P) return;
  const double v = n2[c];
  const bool bad = !(v > tol * ref2[c]) || !(v > 0.0);
  const double nn = bad ? 0.0 : sqrt(v);
  const double nj = nu[(int64_t)j * P + c];
  nu[(int64_t)(j + 1) * P + c] = nn;
  Hb[(int64_t)c * hstride + (int64_t)j * ldh + j + 1] = c128{nj > 0.0 ? nn / nj : 0.0, 0.0};
  flag[c] = bad ? 1 : 0;
}
void launch_lazy_next(int P, int j, const double* n2, const double* ref2, double tol, double* nu, c128* Hb, int ldh,
                      int64_t hstride, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_lazy_next, dim3((P + 63) / 64), dim3(64), 0, s, P, j, n2, ref2, tol, nu, Hb, ldh, hstride,
                     flag);
}
// nu_0 = ||r||, S = nu_0 (first LS block), inactive/zero columns flagged.
__global__ void k_lazy_start(int P, const double* __restrict__ r2, double* __restrict__ nu, c128* __restrict__ S,
                             int* __restrict__ flag) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P) return;
  const double n = r2[c] > 0.0 ? sqrt(r2[c]) : 0.0;
  nu[c] = n;
  S[c] = c128{n, 0.0};
  flag[c] = n > 0.0 ? 0 : 1;
}
void launch_lazy_start(int P, const double* r2, double* nu, c128* S, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_lazy_start, dim3((P + 63) / 64), dim3(64), 0, s, P, r2, nu, S, flag);
}
// Solution coefficients for the stored z~_i = nu_i z_i: Y[i][c] /= nu_i.
__global__ void k_lazy_y(int P, int k, const double* __restrict__ nu, c128* __restrict__ Y) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= k * P) return;
  const double n = nu[t];
  const double a = n > 0.0 ? 1.0 / n : 0.0;
  Y[t] = c128{Y[t].re * a, Y[t].im * a};
}
void launch_lazy_y(int P, int k, const double* nu, c128* Y, hipStream_t s) {
  hipLaunchKernelGGL(k_lazy_y, dim3((k * P + 255) / 256), dim3(256), 0, s, P, k, nu, Y);
}

// ---------------------------------------------------------------------------
// Fixed-step GMRES of the coarsest grid (one independent GMRES per column).
// ---------------------------------------------------------------------------
// Column j of every column's Hessenberg matrix H[c] ((k+1) x k, column-major)
// from the Gram coefficients Gc[i][c] (i <= j) and ||w||^2; sc[c] = 1/||w||.
__global__ void k_cg_hcol(int P, int j, int k, const c128* __restrict__ Gc, const double* __restrict__ hn2,
                          c128* __restrict__ H, double* __restrict__ sc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P) return;
  c128* h = H + (int64_t)c * (k + 1) * k + (int64_t)j * (k + 1);
  for (int i = 0; i <= j; ++i) h[i] = Gc[(int64_t)i * P + c];
  const double nrm = sqrt(fmax(hn2[c], 0.0));
  h[j + 1] = c128{nrm, 0.0};
  sc[c] = nrm > 0.0 ? 1.0 / nrm : 0.0;
}
void launch_cg_hcol(int P, int j, int k, const c128* Gc, const double* hn2, c128* H, double* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_hcol, dim3((P + 63) / 64), dim3(64), 0, s, P, j, k, Gc, hn2, H, sc);
}
// Lazy normalisation of the coarsest GMRES: the stored basis vector s_i has
// norm nu_i (nu[i P + c]; nu_0 = 1, or 0 for a zero column) and the
// orthonormal basis is v_i = s_i / nu_i. With w = M s_j and G_i = s_i^H w,
// the Hessenberg entries are h_ij = G_i / (nu_i nu_j), and
//   s_{j+1} = (w - sum_i s_i G_i / nu_i^2) / nu_j = M v_j - sum_i v_i h_ij
// has norm h_{j+1,j} = nu_{j+1}: the scaling rides on the update's single
// pass (its output scale) instead of a pass of its own, and the stored
// vectors keep the size of an Arnoldi residual.
__global__ void k_cg_lazy_init(int P, const double* __restrict__ b2, double* __restrict__ nu) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < P) nu[c] = b2[c] > 0.0 ? 1.0 : 0.0;
}
void launch_cg_lazy_init(int P, const double* b2, double* nu, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_lazy_init, dim3((P + 63) / 64), dim3(64), 0, s, P, b2, nu);
}
// Before step j's update: C_i = G_i / nu_i^2 in place (i <= j), osc = 1/nu_j.
__global__ void k_cg_lazy_coef(int P, int j, c128* __restrict__ Gc, const double* __restrict__ nu,
                               double* __restrict__ osc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P) return;
  for (int i = 0; i <= j; ++i) {
    const double ni = nu[(int64_t)i * P + c];
    const double a = ni > 0.0 ? 1.0 / (ni * ni) : 0.0;
    const c128 g = Gc[(int64_t)i * P + c];
    Gc[(int64_t)i * P + c] = c128{a * g.re, a * g.im};
  }
  const double nj = nu[(int64_t)j * P + c];
  osc[c] = nj > 0.0 ? 1.0 / nj : 0.0;
}
void launch_cg_lazy_coef(int P, int j, c128* Gc, const double* nu, double* osc, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_lazy_coef, dim3((P + 63) / 64), dim3(64), 0, s, P, j, Gc, nu, osc);
}
// After it: column j of every column's Hessenberg (layout of k_cg_hcol),
// h_ij = C_i nu_i / nu_j, h_{j+1,j} = nu_{j+1} = sqrt(hn2).
__global__ void k_cg_lazy_hcol(int P, int j, int k, const c128* __restrict__ Gc, const double* __restrict__ hn2,
                               double* __restrict__ nu, c128* __restrict__ H) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P) return;
  c128* h = H + (int64_t)c * (k + 1) * k + (int64_t)j * (k + 1);
  const double nj = nu[(int64_t)j * P + c];
  for (int i = 0; i <= j; ++i) {
    const double a = nj > 0.0 ? nu[(int64_t)i * P + c] / nj : 0.0;
    const c128 g = Gc[(int64_t)i * P + c];
    h[i] = c128{a * g.re, a * g.im};
  }
  const double nn = sqrt(fmax(hn2[c], 0.0));
  h[j + 1] = c128{nn, 0.0};
  nu[(int64_t)(j + 1) * P + c] = nn;
}
void launch_cg_lazy_hcol(int P, int j, int k, const c128* Gc, const double* hn2, double* nu, c128* H,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_cg_lazy_hcol, dim3((P + 63) / 64), dim3(64), 0, s, P, j, k, Gc, hn2, nu, H);
}

// sc[c] = 1/sqrt(b2[c]) (0 for a zero column)
__global__ void k_inv_sqrt(int P, const double* __restrict__ b2, double* __restrict__ sc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < P) sc[c] = b2[c] > 0.0 ? 1.0 / sqrt(b2[c]) : 0.0;
}
void launch_inv_sqrt(int P, const double* b2, double* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_inv_sqrt, dim3((P + 63) / 64), dim3(64), 0, s, P, b2, sc);
}
// Least squares min || beta e1 - H y || per column by Givens rotations;
// y written in update layout Y[i][c] (pb = 1). The rotations are applied in
// place to the column's Hessenberg in global memory (rotation j to rows j,
// j+1 of every later column as soon as it is known) and the rotated
// right-hand side lives in G[i][c]: no per-lane arrays, so the kernel needs no
// scratch memory. Each entry sees the same rotations in the same order as a
// column-by-column sweep.
__global__ void k_cg_ls(int P, int k, c128* __restrict__ Hm, const double* __restrict__ b2, c128* __restrict__ G,
                        c128* __restrict__ Y) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P) return;
  c128* H = Hm + (int64_t)c * (k + 1) * k;  // column j, row i at H[j (k+1) + i]
  const double beta = sqrt(fmax(b2[c], 0.0));
  for (int i = 0; i <= k; ++i) G[(int64_t)i * P + c] = c128{0.0, 0.0};
  G[c] = c128{beta, 0.0};
  int steps = k;
  for (int j = 0; j < k; ++j) {
    const cx<double> a = tcx(H[(int64_t)j * (k + 1) + j]), b = tcx(H[(int64_t)j * (k + 1) + j + 1]);
    const double na = sqrt(a.re * a.re + a.im * a.im), nb = sqrt(b.re * b.re + b.im * b.im);
    const double r = sqrt(na * na + nb * nb);
    if (r == 0.0) {
      steps = j;
      break;
    }
    const cx<double> ph = na > 0.0 ? cx<double>{a.re / na, a.im / na} : cx<double>{1.0, 0.0};
    // [c s; -conj(s) c] with c real and s = ph * conj(b) / r, so that the
    // rotated entry below the diagonal vanishes
    const cx<double> cs = {na / r, 0.0};
    const cx<double> sn = {(ph.re * b.re + ph.im * b.im) / r, (ph.im * b.re - ph.re * b.im) / r};
    const cx<double> msn = {-sn.re, sn.im};
    H[(int64_t)j * (k + 1) + j] = fcx(cx<double>{ph.re * r, ph.im * r});
    for (int l = j + 1; l < k; ++l) {
      c128* col = H + (int64_t)l * (k + 1);
      const cx<double> u = tcx(col[j]), w = tcx(col[j + 1]);
      col[j] = fcx(cs * u + sn * w);
      col[j + 1] = fcx(msn * u + cs * w);
    }
    const cx<double> gj = tcx(G[(int64_t)j * P + c]);
    G[(int64_t)j * P + c] = fcx(cs * gj);
    G[(int64_t)(j + 1) * P + c] = fcx(msn * gj);
    if (nb == 0.0) {  // happy breakdown: exact in this space
      steps = j + 1;
      break;
    }
  }
  for (int i = steps - 1; i >= 0; --i) {
    cx<double> sum = tcx(G[(int64_t)i * P + c]);
    for (int l = i + 1; l < steps; ++l) sum = sum - tcx(H[(int64_t)l * (k + 1) + i]) * tcx(Y[(int64_t)l * P + c]);
    const cx<double> d = tcx(H[(int64_t)i * (k + 1) + i]);
    const double dd = d.re * d.re + d.im * d.im;
    Y[(int64_t)i * P + c] = fcx(cx<double>{(sum.re * d.re + sum.im * d.im) / dd, (sum.im * d.re - sum.re * d.im) / dd});
  }
  for (int i = steps; i < k; ++i) Y[(int64_t)i * P + c] = c128{0.0, 0.0};
}
void launch_cg_ls(int P, int k, c128* H, const double* b2, c128* G, c128* Y, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_ls, dim3((P + 63) / 64), dim3(64), 0, s, P, k, H, b2, G, Y);
}

}  // namespace helm
