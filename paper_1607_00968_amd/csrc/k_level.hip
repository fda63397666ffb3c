// k_level.hip -- per-level kernels of the block multigrid cycle.
//
// Every kernel works on point-major blocks [N][P] (see common.hpp) and lets
// each lane own K consecutive right-hand sides of one grid point, so a
// wavefront reads contiguous runs for the centre and each neighbour.
//
//  - fine level: the 5-point (2D) / 7-point (3D) operator of eq:LinearSystem
//    with a per-point complex diagonal (H or the shifted M) and constant
//    off-diagonals -1/h_a^2;
//  - coarse levels: 9-point / 27-point Galerkin stencils [N][3^d];
//  - damped Jacobi (section 5.3), residual, full-weighting restriction and
//    d-linear prolongation (section "Solving the Helmholtz equation for
//    multiple right hand sides").
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include <hip/hip_cooperative_groups.h>

#include "common.hpp"
#include "kernels.hpp"
#include "tile_gemm.hpp"

namespace helm {

template <class A, class B, class C> constexpr int kmax3() {
  return St<A>::R > St<B>::R ? (St<A>::R > St<C>::R ? St<A>::R : St<C>::R)
                             : (St<B>::R > St<C>::R ? St<B>::R : St<C>::R);
}
__device__ inline void put1(c128* p, c128 v) { *p = v; }
__device__ inline void put1(c64* p, c128 v) { *p = c64{(float)v.re, (float)v.im}; }
__device__ inline void put1(cbf* p, c128 v) { *p = cbf{f2bf((float)v.re), f2bf((float)v.im)}; }
__device__ inline c128 get1(const c128* p) { return *p; }
__device__ inline c128 get1(const c64* p) { return c128{(double)p->re, (double)p->im}; }
__device__ inline c128 get1(const cbf* p) { return c128{(double)bf2f(p->re), (double)bf2f(p->im)}; }

template <int K, class S, class T> __device__ inline void ldK(const S* p, cx<T>* o) {
#pragma unroll
  for (int k = 0; k < K; k += St<S>::R) ld16<T>(p + k, o + k);
}
template <int K, class S, class T> __device__ inline void ldKz(const S* p, bool ok, cx<T>* o) {
  if (ok) {
    ldK<K, S, T>(p, o);
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) o[k] = {(T)0, (T)0};
  }
}
template <int K, class S, class T> __device__ inline void stK(S* p, const cx<T>* o) {
#pragma unroll
  for (int k = 0; k < K; k += St<S>::R) st16<T>(p + k, o + k);
}

// ---------------------------------------------------------------------------
// Fine-level operator family.
//   APPLY : out = A u
//   RESID : out = f - A u
//   JAC   : out = u + w D^-1 (f - A u)      (dw = w / diag)
//   JAC0  : out = w D^-1 f                  (first sweep from u = 0)
// ---------------------------------------------------------------------------
// One work item (K columns of one point) of the fine-level family; the
// kernels below and the persistent cycle both run it, t < npts * P / K.
template <int DIM, class SU, class SF, class SO, class T, int MODE>
__device__ __forceinline__ void fine_item(const Geo& g, int64_t t, const SU* __restrict__ u,
                                          const SF* __restrict__ f, SO* __restrict__ out,
                                          const cx<T>* __restrict__ dg, const cx<T>* __restrict__ dw, T ihx, T ihy,
                                          T ihz) {
  constexpr int K = kmax3<SU, SF, SO>();
  const int Pc = g.P / K;
  const int64_t i = t / Pc;
  const int c = (int)(t - i * Pc) * K;
  const int64_t base = i * g.P + c;
  cx<T> res[K];
  if (MODE == 3) {
    cx<T> fv[K];
    ldK<K, SF, T>(f + base, fv);
    cx<T> w = dw[i];
#pragma unroll
    for (int k = 0; k < K; ++k) res[k] = w * fv[k];
    stK<K, SO, T>(out + base, res);
    return;
  }
  int x, y, z;
  coords(g, i, x, y, z);
  cx<T> uc[K], nb[K], acc[K];
  ldK<K, SU, T>(u + base, uc);
  const cx<T> d = dg[i];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = d * uc[k];
  const int64_t sx = g.P, sy = (int64_t)g.nx * g.P, sz = (int64_t)g.nx * g.ny * g.P;
  // -1/h^2 couplings to the 2*DIM face neighbours (zero outside the grid)
  cx<T> sum[K];
#pragma unroll
  for (int k = 0; k < K; ++k) sum[k] = {(T)0, (T)0};
  ldKz<K, SU, T>(u + base - sx, x > 0, nb);
#pragma unroll
  for (int k = 0; k < K; ++k) sum[k] = sum[k] + ihx * nb[k];
  ldKz<K, SU, T>(u + base + sx, x < g.nx - 1, nb);
#pragma unroll
  for (int k = 0; k < K; ++k) sum[k] = sum[k] + ihx * nb[k];
  ldKz<K, SU, T>(u + base - sy, y > 0, nb);
#pragma unroll
  for (int k = 0; k < K; ++k) sum[k] = sum[k] + ihy * nb[k];
  ldKz<K, SU, T>(u + base + sy, y < g.ny - 1, nb);
#pragma unroll
  for (int k = 0; k < K; ++k) sum[k] = sum[k] + ihy * nb[k];
  if (DIM == 3) {
    ldKz<K, SU, T>(u + base - sz, z > 0, nb);
#pragma unroll
    for (int k = 0; k < K; ++k) sum[k] = sum[k] + ihz * nb[k];
    ldKz<K, SU, T>(u + base + sz, z < g.nz - 1, nb);
#pragma unroll
    for (int k = 0; k < K; ++k) sum[k] = sum[k] + ihz * nb[k];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = acc[k] - sum[k];
  if (MODE == 0) {
    stK<K, SO, T>(out + base, acc);
    return;
  }
  cx<T> fv[K];
  ldK<K, SF, T>(f + base, fv);
  if (MODE == 1) {
#pragma unroll
    for (int k = 0; k < K; ++k) res[k] = fv[k] - acc[k];
  } else {
    const cx<T> w = dw[i];
#pragma unroll
    for (int k = 0; k < K; ++k) res[k] = uc[k] + w * (fv[k] - acc[k]);
  }
  stK<K, SO, T>(out + base, res);
}

template <int DIM, class SU, class SF, class SO, class T, int MODE>
__global__ __launch_bounds__(256) void k_fine(Geo g, const SU* __restrict__ u, const SF* __restrict__ f,
                                              SO* __restrict__ out, const cx<T>* __restrict__ dg,
                                              const cx<T>* __restrict__ dw, T ihx, T ihy, T ihz) {
  constexpr int K = kmax3<SU, SF, SO>();
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.npts * (g.P / K)) return;
  fine_item<DIM, SU, SF, SO, T, MODE>(g, t, u, f, out, dg, dw, ihx, ihy, ihz);
}

// ---------------------------------------------------------------------------
// 3D fine-level operator, z-marching: each lane owns K columns of one (x, y)
// grid column and walks a chunk of z planes, keeping u(z-1), u(z), u(z+1) in
// registers, so every value of u is fetched from memory once; the in-plane
// neighbours come from L1/L2. Workgroups are numbered so that each XCD (the
// hardware deals workgroup b to XCD b % 8) receives a contiguous run of
// tiles ordered y-fastest: tiles of neighbouring y rows run at the same time
// on the same XCD and share its L2. Same modes as k_fine except JAC0.
// ---------------------------------------------------------------------------
struct ZTiles {
  int nxb, nzc, zc;  // x-blocks, z-chunks, planes per chunk
  int per;           // tiles per XCD
  int64_t ntiles;
};

template <class SU, class SF, class SO, class T, int MODE, int RY>
__global__ __launch_bounds__(256) void k_fine_zm(Geo g, ZTiles zt, const SU* __restrict__ u,
                                                 const SF* __restrict__ f, SO* __restrict__ out,
                                                 const cx<T>* __restrict__ dg, const cx<T>* __restrict__ dw, T ihx,
                                                 T ihy, T ihz) {
  constexpr int K = kmax3<SU, SF, SO>();
  const int L = g.P / K;      // lanes per point
  const int PPB = 256 / L;    // points per workgroup along x
  const int lane = threadIdx.x % L, px = threadIdx.x / L;
  const int64_t t = (int64_t)(blockIdx.x % 8) * zt.per + blockIdx.x / 8;
  if (t >= zt.ntiles || px >= PPB) return;
  const int nyb = (g.ny + RY - 1) / RY;
  const int yb = (int)(t % nyb);
  const int xb = (int)((t / nyb) % zt.nxb);
  const int zc = (int)(t / ((int64_t)nyb * zt.nxb));
  const int x = xb * PPB + px;
  if (x >= g.nx) return;
  const int y0 = yb * RY;
  const int ry = g.ny - y0 < RY ? g.ny - y0 : RY;  // rows of this tile
  const int z0 = zc * zt.zc;
  const int z1 = z0 + zt.zc < g.nz ? z0 + zt.zc : g.nz;
  const int c = lane * K;
  const int64_t sx = g.P, sy = (int64_t)g.nx * g.P, sz = (int64_t)g.nx * g.ny * g.P;
  const int64_t plane = (int64_t)g.nx * g.ny;
  int64_t i = ((int64_t)z0 * g.ny + y0) * g.nx + x;  // point (x, y0, z)
  const SU* up = u + i * g.P + c;
  // rows r >= ry never load and never store (values stay zero)
  cx<T> um[RY][K], uc[RY][K], un[RY][K], nb[K];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    ldKz<K, SU, T>(up + r * sy - sz, r < ry && z0 > 0, um[r]);
    ldKz<K, SU, T>(up + r * sy, r < ry, uc[r]);
  }
  for (int z = z0; z < z1; ++z, i += plane, up += sz) {
#pragma unroll
    for (int r = 0; r < RY; ++r) ldKz<K, SU, T>(up + r * sy + sz, r < ry && z + 1 < g.nz, un[r]);
    cx<T> lo[K], hi[K];  // y-halo rows y0-1 and y0+ry
    ldKz<K, SU, T>(up - sy, y0 > 0, lo);
    ldKz<K, SU, T>(up + ry * sy, y0 + ry < g.ny, hi);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      if (r >= ry) break;
      const int64_t ir = i + (int64_t)r * g.nx;
      const cx<T> d = dg[ir];
      cx<T> acc[K], sum[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        acc[k] = d * uc[r][k];
        const cx<T> ylo = r == 0 ? lo[k] : uc[r > 0 ? r - 1 : 0][k];
        const cx<T> yhi = r == ry - 1 ? hi[k] : uc[r + 1 < RY ? r + 1 : r][k];
        sum[k] = ihz * (um[r][k] + un[r][k]) + ihy * (ylo + yhi);
      }
      ldKz<K, SU, T>(up + r * sy - sx, x > 0, nb);
#pragma unroll
      for (int k = 0; k < K; ++k) sum[k] = sum[k] + ihx * nb[k];
      ldKz<K, SU, T>(up + r * sy + sx, x < g.nx - 1, nb);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        sum[k] = sum[k] + ihx * nb[k];
        acc[k] = acc[k] - sum[k];
      }
      const int64_t o = ir * g.P + c;
      if (MODE == 0) {
        stK<K, SO, T>(out + o, acc);
      } else {
        cx<T> fv[K], res[K];
        ldK<K, SF, T>(f + o, fv);
        if (MODE == 1) {
#pragma unroll
          for (int k = 0; k < K; ++k) res[k] = fv[k] - acc[k];
        } else {
          const cx<T> w = dw[ir];
#pragma unroll
          for (int k = 0; k < K; ++k) res[k] = uc[r][k] + w * (fv[k] - acc[k]);
        }
        stK<K, SO, T>(out + o, res);
      }
    }
#pragma unroll
    for (int r = 0; r < RY; ++r)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        um[r][k] = uc[r][k];
        uc[r][k] = un[r][k];
      }
  }
}

// ---------------------------------------------------------------------------
// Galerkin-level operator family (same modes), stencil [N][NS], NS = 3^DIM.
// ---------------------------------------------------------------------------
template <int DIM, class S, class T, int MODE>
__device__ __forceinline__ void gal_item(const Geo& g, int64_t t, const S* __restrict__ u, const S* __restrict__ f,
                                         S* __restrict__ out, const cx<T>* __restrict__ st,
                                         const cx<T>* __restrict__ dw) {
  constexpr int K = St<S>::R;
  constexpr int NS = DIM == 3 ? 27 : 9;
  const int Pc = g.P / K;
  const int64_t i = t / Pc;
  const int c = (int)(t - i * Pc) * K;
  const int64_t base = i * g.P + c;
  cx<T> res[K];
  if (MODE == 3) {
    cx<T> fv[K];
    ldK<K, S, T>(f + base, fv);
    const cx<T> w = dw[i];
#pragma unroll
    for (int k = 0; k < K; ++k) res[k] = w * fv[k];
    stK<K, S, T>(out + base, res);
    return;
  }
  int x, y, z;
  coords(g, i, x, y, z);
  cx<T> acc[K], nb[K], uc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = {(T)0, (T)0};
  const cx<T>* sp = st + i * NS;
  // one stencil entry per iteration, unrolled by 3 only: bounds the
  // number of neighbour loads in flight (and so the registers they hold)
#pragma unroll 3
  for (int o = 0; o < NS; ++o) {
    const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = DIM == 3 ? o / 9 - 1 : 0;
    const bool ok = (x + ox >= 0) && (x + ox < g.nx) && (y + oy >= 0) && (y + oy < g.ny) && (z + oz >= 0) &&
                    (z + oz < g.nz);
    const int64_t off = (((int64_t)oz * g.ny + oy) * g.nx + ox) * g.P;
    ldKz<K, S, T>(u + base + off, ok, nb);
    if (o == NS / 2) {
#pragma unroll
      for (int k = 0; k < K; ++k) uc[k] = nb[k];
    }
    const cx<T> a = sp[o];
#pragma unroll
    for (int k = 0; k < K; ++k) cfma(acc[k], a, nb[k]);
  }
  if (MODE == 0) {
    stK<K, S, T>(out + base, acc);
    return;
  }
  cx<T> fv[K];
  ldK<K, S, T>(f + base, fv);
  if (MODE == 1) {
#pragma unroll
    for (int k = 0; k < K; ++k) res[k] = fv[k] - acc[k];
  } else {
    const cx<T> w = dw[i];
#pragma unroll
    for (int k = 0; k < K; ++k) res[k] = uc[k] + w * (fv[k] - acc[k]);
  }
  stK<K, S, T>(out + base, res);
}

template <int DIM, class S, class T, int MODE>
__global__ __launch_bounds__(256) void k_gal(Geo g, const S* __restrict__ u, const S* __restrict__ f,
                                             S* __restrict__ out, const cx<T>* __restrict__ st,
                                             const cx<T>* __restrict__ dw) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.npts * (g.P / St<S>::R)) return;
  gal_item<DIM, S, T, MODE>(g, t, u, f, out, st, dw);
}

// ---------------------------------------------------------------------------
// Full weighting: rc[I] = 2^-d sum_delta w(delta) rf[2I+1+delta],
// w = prod over axes of (1 if delta_a == 0 else 1/2).
// ---------------------------------------------------------------------------
template <int DIM, class SI, class SO, class T>
__device__ __forceinline__ void restrict_item(const Geo& gf, const Geo& gc, int64_t t, const SI* __restrict__ rf,
                                              SO* __restrict__ rc) {
  constexpr int K = St<SI>::R > St<SO>::R ? St<SI>::R : St<SO>::R;
  const int Pc = gc.P / K;
  const int64_t I = t / Pc;
  const int c = (int)(t - I * Pc) * K;
  int X, Y, Z;
  coords(gc, I, X, Y, Z);
  cx<T> acc[K], v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = {(T)0, (T)0};
  const int zlo = DIM == 3 ? -1 : 0, zhi = DIM == 3 ? 1 : 0;
#pragma unroll
  for (int dz = zlo; dz <= zhi; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int fx = 2 * X + 1 + dx, fy = 2 * Y + 1 + dy, fz = DIM == 3 ? 2 * Z + 1 + dz : 0;
        const T w = (dx ? (T)0.5 : (T)1) * (dy ? (T)0.5 : (T)1) * (dz ? (T)0.5 : (T)1);
        const int64_t fi = ((int64_t)fz * gf.ny + fy) * gf.nx + fx;
        ldK<K, SI, T>(rf + fi * gf.P + c, v);
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] = acc[k] + w * v[k];
      }
  const T s = DIM == 3 ? (T)0.125 : (T)0.25;
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = s * acc[k];
  stK<K, SO, T>(rc + I * gc.P + c, acc);
}

template <int DIM, class SI, class SO, class T>
__global__ __launch_bounds__(256) void k_restrict(Geo gf, Geo gc, const SI* __restrict__ rf, SO* __restrict__ rc) {
  constexpr int K = St<SI>::R > St<SO>::R ? St<SI>::R : St<SO>::R;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= gc.npts * (gc.P / K)) return;
  restrict_item<DIM, SI, SO, T>(gf, gc, t, rf, rc);
}

// ---------------------------------------------------------------------------
// Prolongation and correction: uf += P ec. A fine index i has the coarse
// parent (i-1)/2 with weight 1 when i is odd, else the parents i/2-1 and i/2
// (those inside the coarse grid) with weight 1/2.
// ---------------------------------------------------------------------------
__device__ inline int parents(int i, int nc, int* p, float* w) {
  if (i & 1) {
    p[0] = (i - 1) >> 1;
    w[0] = 1.f;
    return 1;
  }
  int k = 0;
  if (i / 2 - 1 >= 0) {
    p[k] = i / 2 - 1;
    w[k++] = 0.5f;
  }
  if (i / 2 < nc) {
    p[k] = i / 2;
    w[k++] = 0.5f;
  }
  return k;
}

template <int DIM, class SC, class SF, class T>
__device__ __forceinline__ void prolong_item(const Geo& gf, const Geo& gc, int64_t t, const SC* __restrict__ ec,
                                             SF* __restrict__ uf) {
  constexpr int K = St<SC>::R > St<SF>::R ? St<SC>::R : St<SF>::R;
  const int Pc = gf.P / K;
  const int64_t i = t / Pc;
  const int c = (int)(t - i * Pc) * K;
  int x, y, z;
  coords(gf, i, x, y, z);
  int px[2], py[2], pz[2] = {0, 0};
  float wx[2], wy[2], wz[2] = {1.f, 1.f};
  const int nx = parents(x, gc.nx, px, wx);
  const int ny = parents(y, gc.ny, py, wy);
  const int nz = DIM == 3 ? parents(z, gc.nz, pz, wz) : 1;
  cx<T> acc[K], v[K];
  ldK<K, SF, T>(uf + i * gf.P + c, acc);
  for (int a = 0; a < nz; ++a)
    for (int b = 0; b < ny; ++b)
      for (int e = 0; e < nx; ++e) {
        const T w = (T)(wx[e] * wy[b] * wz[a]);
        const int64_t ci = ((int64_t)pz[a] * gc.ny + py[b]) * gc.nx + px[e];
        ldK<K, SC, T>(ec + ci * gc.P + c, v);
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] = acc[k] + w * v[k];
      }
  stK<K, SF, T>(uf + i * gf.P + c, acc);
}

template <int DIM, class SC, class SF, class T>
__global__ __launch_bounds__(256) void k_prolong_add(Geo gf, Geo gc, const SC* __restrict__ ec, SF* __restrict__ uf) {
  constexpr int K = St<SC>::R > St<SF>::R ? St<SC>::R : St<SF>::R;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= gf.npts * (gf.P / K)) return;
  prolong_item<DIM, SC, SF, T>(gf, gc, t, ec, uf);
}

// ---------------------------------------------------------------------------
// Layout and precision conversion.
// ---------------------------------------------------------------------------
template <class SI, class SO, class T>
__global__ __launch_bounds__(256) void k_convert(int64_t nvec, const SI* __restrict__ a, SO* __restrict__ b) {
  constexpr int K = St<SI>::R > St<SO>::R ? St<SI>::R : St<SO>::R;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t * K >= nvec) return;
  cx<T> v[K];
  ldK<K, SI, T>(a + t * K, v);
  stK<K, SO, T>(b + t * K, v);
}

// ABI [nrhs][N] complex128 -> internal [N][P] (columns >= nrhs zeroed).
template <class SO>
__global__ __launch_bounds__(256) void k_to_internal(int64_t N, int nrhs, int P, const c128* __restrict__ src,
                                                     SO* __restrict__ dst) {
  __shared__ c128 tile[32][33];
  const int64_t n0 = (int64_t)blockIdx.x * 32;
  const int s0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int s = s0 + r;
    const int64_t n = n0 + tx;
    tile[r][tx] = (s < nrhs && n < N) ? src[(int64_t)s * N + n] : c128{0.0, 0.0};
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t n = n0 + r;
    const int s = s0 + tx;
    if (n < N && s < P) put1(dst + n * P + s, tile[tx][r]);
  }
}

// internal [N][P] -> ABI [nrhs][N] complex128.
template <class SI>
__global__ __launch_bounds__(256) void k_to_abi(int64_t N, int nrhs, int P, const SI* __restrict__ src,
                                                c128* __restrict__ dst) {
  __shared__ c128 tile[32][33];
  const int64_t n0 = (int64_t)blockIdx.x * 32;
  const int s0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int64_t n = n0 + r;
    const int s = s0 + tx;
    c128 v{0.0, 0.0};
    if (n < N && s < P) v = get1(src + n * P + s);
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int s = s0 + r;
    const int64_t n = n0 + tx;
    if (s < nrhs && n < N) dst[(int64_t)s * N + n] = tile[tx][r];
  }
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
static inline dim3 grid1(int64_t threads) { return dim3((unsigned)((threads + 255) / 256)); }

// Tile shape of the 3D marching kernel (set by the host's autotuner):
// y rows per lane and z planes per chunk. Every shape computes each output
// from the same loads in the same order, so results are bitwise identical.
// ---------------------------------------------------------------------------
// 3D fine-level operator, 2.5D blocking through LDS: a workgroup of 64*TY
// lanes owns a 16 x TY tile of grid columns (TY = 16 or 8) for one group of
// CG right-hand sides (128 B per point: 16 complex64 or 8 complex128) and
// walks a chunk of z planes. Lane (point q, slot sl) keeps u(z-1), u(z+1) of
// its CG/4 columns in registers; plane z of the tile and its one-point ring
// are staged in LDS, so every in-plane neighbour comes from LDS and u is read
// from memory (18 (TY+2)) / (16 TY) times per plane (1.27 at TY = 16, 1.41 at
// TY = 8) instead of once per neighbouring tile in L2. The sums are formed in
// the order of k_fine_zm, so the results are bitwise those of every other
// tile shape. Modes APPLY, RESID, JAC.
// ---------------------------------------------------------------------------
constexpr int TB = 16;  // tile edge along x (points)

template <class T, class E> __device__ inline cx<T> wid(const cx<E>& v) { return cx<T>{(T)v.re, (T)v.im}; }

// Parents of fine index i along one axis in registers (the order and weights
// of parents(): the lower parent first).
struct Par {
  int p0, p1, n;
  float w0, w1;
};
__device__ inline Par par_of(int i, int nc) {
  Par r;
  if (i & 1) {
    r.p0 = (i - 1) >> 1;
    r.w0 = 1.f;
    r.p1 = r.p0;
    r.w1 = 0.f;
    r.n = 1;
    return r;
  }
  const bool lo = i / 2 - 1 >= 0, hi = i / 2 < nc;
  r.p0 = lo ? i / 2 - 1 : i / 2;
  r.p1 = i / 2;
  r.w0 = r.w1 = 0.5f;
  r.n = (lo ? 1 : 0) + (hi ? 1 : 0);
  return r;
}

// The sweep's input u at fine point (x, y, z), K columns from p:
//  PRO = 0: u as stored;
//  PRO = 1: u with the coarse-grid correction added on the fly, u + P e, the
//           terms in the order of k_prolong_add;
//  PRO = 2: p points at f and u is the zero-guess sweep's result w D^-1 f,
//           formed as that sweep forms it (so the fused pair of sweeps is
//           bitwise the two separate ones).
// Coarse correction staged in LDS for the prolongation-fused sweep: a window
// of LCZ coarse planes (slot = plane % LCZ) of the LCX x LCY coarse points
// the 16 x TY fine tile and its ring interpolate from, CG columns each.
struct LCoarse {
  const unsigned char* base;  // LDS, this lane's K columns of point 0 of slot 0
  int cx0, cy0;               // coarse (x, y) of the window's first point
  int stride_pt, stride_slot; // bytes between points / between plane slots
};
constexpr int LCZ = 3;

template <int K, class S, class SC, class T, int PRO, bool LDSC = false>
__device__ inline void ld_u(const S* p, bool ok, int x, int y, int z, const SC* ec, const Geo& gc,
                            const cx<T>* dwp, int64_t pt, int c, cx<T>* o, const LCoarse& lc = LCoarse{}) {
  ldKz<K, S, T>(p, ok, o);
  if (PRO == 2) {
    if (ok) {
      const cx<T> w = dwp[pt];  // pt: the point's index (z, y, x)
#pragma unroll
      for (int k = 0; k < K; ++k) o[k] = w * o[k];
    }
    return;
  }
  if (!PRO || !ok) return;
  if (LDSC) {
    // recompute the (loop-invariant) parents of x and y at every use: a few
    // integer operations, where keeping them for the own point and the ring
    // point would hold about 20 registers through the whole z march
    asm volatile("" : "+v"(x), "+v"(y));
  }
  const Par ax = par_of(x, gc.nx), ay = par_of(y, gc.ny), az = par_of(z, gc.nz);
  cx<T> v[K];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    if (a >= az.n) break;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      if (b >= ay.n) break;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        if (e >= ax.n) break;
        const float wx = e ? ax.w1 : ax.w0, wy = b ? ay.w1 : ay.w0, wz = a ? az.w1 : az.w0;
        const T w = (T)(wx * wy * wz);
        const int cx_ = e ? ax.p1 : ax.p0, cy_ = b ? ay.p1 : ay.p0, cz_ = a ? az.p1 : az.p0;
        if (LDSC) {
          const unsigned char* q = lc.base + (cz_ % LCZ) * lc.stride_slot +
                                   ((cy_ - lc.cy0) * (TB / 2 + 2) + (cx_ - lc.cx0)) * lc.stride_pt;
          ldK<K, SC, T>(reinterpret_cast<const SC*>(q), v);
        } else {
          const int64_t ci = ((int64_t)cz_ * gc.ny + cy_) * gc.nx + cx_;
          ldK<K, SC, T>(ec + ci * gc.P + c, v);
        }
#pragma unroll
        for (int k = 0; k < K; ++k) o[k] = o[k] + w * v[k];
        // LDS parents one at a time: the scheduler would otherwise hoist all
        // eight reads (8 x 2K registers) ahead of their sums
        if (LDSC) __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
}

template <class S, class T, int MODE, int TY, class SC = S, int PRO = 0>
__global__ __launch_bounds__(64 * TY) void k_fine_t16(Geo g, ZTiles zt, int nyb, const S* __restrict__ u,
                                                      const S* __restrict__ f, S* __restrict__ out,
                                                      const cx<T>* __restrict__ dg, const cx<T>* __restrict__ dw,
                                                      T ihx, T ihy, T ihz, const SC* __restrict__ ec, Geo gc) {
  constexpr int CG = 128 / (int)sizeof(S);  // columns per group
  constexpr int K = CG / 4;                  // columns per lane
  constexpr int HX = TB + 2, HY = TY + 2;
  constexpr int RING = 2 * HX + 2 * TY;     // ring points
  // Slot-major LDS: the 32 B of a lane's columns for point p sit at
  // sm_slot[sl] + 32 p, with the four slot planes 256-B aligned plus 0, 16,
  // 128, 144 B, so the 16 lanes of one 128-bit LDS pass (4 points x 4 slots)
  // hit 16 distinct 16-B bank groups.
  constexpr int NPT = HX * HY;
  constexpr int PSR = (NPT * 32 + 255) / 256 * 256;
  __shared__ __attribute__((aligned(256))) unsigned char smraw[4 * PSR + 256];
  // PRO = 1 with BF16 coarse fields on 16-row tiles: the coarse correction
  // the tile interpolates from is staged in LDS one coarse plane at a time
  // (16 B = K columns per chunk), instead of every fine value gathering its
  // up to 8 parents from global memory
  constexpr bool LDSC = PRO == 1 && TY == 16 && sizeof(SC) * K == 16;
  constexpr int LCX = TB / 2 + 2, LCY = TY / 2 + 2;
  constexpr int LPT = CG * (int)sizeof(SC);  // bytes per coarse point
  constexpr int LSLOT = LCX * LCY * LPT;
  __shared__ __attribute__((aligned(16))) unsigned char lcraw[LDSC ? LCZ * LSLOT : 16];
  const int64_t t0 = (int64_t)(blockIdx.x % 8) * zt.per + blockIdx.x / 8;
  if (t0 >= zt.ntiles) return;  // whole workgroup leaves together
  int64_t t = t0;
  const int yb = (int)(t % nyb);
  t /= nyb;
  const int xb = (int)(t % zt.nxb);
  t /= zt.nxb;
  const int zc = (int)(t % zt.nzc);
  const int cgi = (int)(t / zt.nzc);
  const int q = threadIdx.x >> 2, sl = threadIdx.x & 3;
  const int px = q % TB, py = q / TB;
  const int x = xb * TB + px, y = yb * TY + py;
  const bool inb = x < g.nx && y < g.ny;
  const int c = cgi * CG + sl * K;
  const int z0 = zc * zt.zc;
  const int z1 = z0 + zt.zc < g.nz ? z0 + zt.zc : g.nz;
  const int64_t plane = (int64_t)g.nx * g.ny, sz = plane * g.P;
  // ring point of this lane (lanes 0 .. 4*RING-1): halo coordinates (hx, hy)
  const int rp = threadIdx.x >> 2;
  int hx, hy;
  if (rp < HX) {
    hx = rp;
    hy = 0;
  } else if (rp < 2 * HX) {
    hx = rp - HX;
    hy = HY - 1;
  } else if (rp < 2 * HX + TY) {
    hx = 0;
    hy = rp - 2 * HX + 1;
  } else {
    hx = HX - 1;
    hy = rp - 2 * HX - TY + 1;
  }
  const int rx = xb * TB + hx - 1, ry = yb * TY + hy - 1;
  const bool ring = rp < RING;
  const bool rin = ring && rx >= 0 && rx < g.nx && ry >= 0 && ry < g.ny;
  const int64_t icol = (int64_t)y * g.nx + x;    // own (x, y) column index
  const int64_t rcol = (int64_t)ry * g.nx + rx;  // ring (x, y) column index
  LCoarse lc;
  lc.base = lcraw + sl * 16;
  lc.cx0 = xb * (TB / 2) - 1;
  lc.cy0 = yb * (TY / 2) - 1;
  lc.stride_pt = LPT;
  lc.stride_slot = LSLOT;
  // coarse plane pz (all window points, zero outside the coarse grid) into
  // slot pz % LCZ: the global load now, the LDS store by put_stage later
  uint4 stv = {0u, 0u, 0u, 0u};
  int stpz = -1;
  const int ste = threadIdx.x;  // chunk of this lane (LCX * LCY * 4 chunks)
  auto load_stage = [&](int pz) {
    stpz = -1;
    if (!LDSC || pz < 0 || pz >= gc.nz || ste >= LCX * LCY * 4) return;
    stpz = pz;
    const int pi = ste >> 2, q = ste & 3;
    const int ccx = lc.cx0 + pi % LCX, ccy = lc.cy0 + pi / LCX;
    stv = uint4{0u, 0u, 0u, 0u};
    if (ccx >= 0 && ccx < gc.nx && ccy >= 0 && ccy < gc.ny)
      stv = *reinterpret_cast<const uint4*>(ec + (((int64_t)pz * gc.ny + ccy) * gc.nx + ccx) * gc.P + cgi * CG + q * K);
  };
  auto put_stage = [&]() {
    if (!LDSC || stpz < 0) return;
    *reinterpret_cast<uint4*>(lcraw + (stpz % LCZ) * LSLOT + (ste >> 2) * LPT + (ste & 3) * 16) = stv;
  };
  if (LDSC) {
    // the window the prologue and the first step read: the parents of
    // planes z0 - 1 (if it exists) to z0 + 1
    const int zl = z0 > 0 ? z0 - 1 : z0;
    const int plo = ((zl & 1) ? zl / 2 : zl / 2 - 1) < 0 ? 0 : ((zl & 1) ? zl / 2 : zl / 2 - 1);
    const int phi = (z0 + 1) / 2 < gc.nz - 1 ? (z0 + 1) / 2 : gc.nz - 1;
    for (int pz = plo; pz <= phi; ++pz) {
      load_stage(pz);
      put_stage();
    }
    __syncthreads();
  }
  // TY = 8 prefetches one plane ahead (u(z+2), the ring of z+1, f(z+1) are
  // in flight while plane z is computed); TY = 16 keeps the registers low
  constexpr bool PF = TY == 8;
  cx<T> um[K], uc[K], un[K], unn[K], rc[K], rn[K], fc[K], fn[K];
  // PRO = 2 reads u from f (the zero-guess sweep is formed on the fly):
  // the same pointers, so that the compiler keeps one copy of them
  const S* ub = PRO == 2 ? f : u;
  const S* up = ub + ((int64_t)z0 * plane + icol) * g.P + c;
  const S* rpp = ub + ((int64_t)z0 * plane + rcol) * g.P + c;
  const S* fp = f + ((int64_t)z0 * plane + icol) * g.P + c;
  // RAWC (PRO = 2): the own column keeps f itself at z and z + 1 (uc, un)
  // with the point's w D^-1 (wc, wn; 0 outside the grid), loaded one plane
  // ahead, and the zero-guess sweep's value w D^-1 f at z - 1 (um). That
  // value is formed where it is used (the same product ld_u forms, so the
  // results are unchanged), and f(z) needs no second load.
  constexpr bool RAWC = PRO == 2 && !PF;
  cx<T> wc{}, wn{};
  if (RAWC) {
    ld_u<K, S, SC, T, PRO, LDSC>(up - sz, inb && z0 > 0, x, y, z0 - 1, ec, gc, dw,
                                 (int64_t)(z0 - 1) * plane + icol, c, um, lc);
    ldKz<K, S, T>(up, inb, uc);
    if (inb) wc = dw[(int64_t)z0 * plane + icol];
  } else {
    ld_u<K, S, SC, T, PRO, LDSC>(up - sz, inb && z0 > 0, x, y, z0 - 1, ec, gc, dw,
                                 (int64_t)(z0 - 1) * plane + icol, c, um, lc);
    ld_u<K, S, SC, T, PRO, LDSC>(up, inb, x, y, z0, ec, gc, dw, (int64_t)z0 * plane + icol, c, uc, lc);
  }
  if (PF) {
    ld_u<K, S, SC, T, PRO>(up + sz, inb && z0 + 1 < g.nz, x, y, z0 + 1, ec, gc, dw, (int64_t)(z0 + 1) * plane + icol,
                           c, un);
    ld_u<K, S, SC, T, PRO>(rpp, rin, rx, ry, z0, ec, gc, dw, (int64_t)z0 * plane + rcol, c, rc);
    if (MODE != 0) ldKz<K, S, T>(fp, inb, fc);
  }
  // the tile holds values in storage precision (32 B per lane and point);
  // widening them to T on the way out of LDS is exact
  using LE = typename std::conditional<sizeof(S) == 8, float, double>::type;
  cx<LE>* sm = reinterpret_cast<cx<LE>*>(smraw + sl * PSR + (sl & 1) * 16 + (sl >> 1) * 128);
  const int me = ((py + 1) * HX + px + 1) * K;  // own point, in units of cx<LE>
  const int ro = (hy * HX + hx) * K;
  constexpr int RX = K, RYS = HX * K;           // x and y neighbour strides
  // One base address for the own point and its four in-plane neighbours:
  // the lowest of them (y - 1), so that every access is the base plus a
  // constant non-negative offset (LDS offsets cannot be negative). The empty
  // asm keeps the compiler from folding the base back into `me` and holding
  // separate address registers for the neighbours below it.
  int lo = me - RYS;
  asm volatile("" : "+v"(lo));
  cx<LE>* const nb = sm + lo;
  // When each plane's other operands are issued (loads complete in issue
  // order, so an operand issued before the u loads is waited for with them):
  //  EF: f, D and w D^-1 right after the plane's LDS stores, so that their
  //      latency overlaps the barrier (sweeps and residuals; measured at
  //      192^3 x 64: the plain sweep 2.45 -> 2.25 ms, the prolongation-fused
  //      one 2.42 -> 2.32 ms; issued with the u loads instead, the fused one
  //      took 2.63 ms);
  //  EF2: D ahead of the u loads (RAWC, which needs neither f nor w D^-1
  //      after the barrier: nothing is loaded there; 1.82 -> 1.76 ms; and
  //      the operator apply, which has no f).
  constexpr bool EF = !RAWC && !PF && MODE != 0;
  constexpr bool EF2 = RAWC || (MODE == 0 && !PF);
  for (int z = z0; z < z1; ++z, up += sz, rpp += sz, fp += sz) {
    cx<T> de{}, we{};
    if (EF2 && inb) de = dg[(int64_t)z * plane + icol];
    if (PF) {
      const bool more = z + 1 < z1;
      ld_u<K, S, SC, T, PRO>(up + 2 * sz, inb && z + 2 < g.nz, x, y, z + 2, ec, gc, dw,
                             (int64_t)(z + 2) * plane + icol, c, unn);
      ld_u<K, S, SC, T, PRO>(rpp + sz, rin && more, rx, ry, z + 1, ec, gc, dw, (int64_t)(z + 1) * plane + rcol, c,
                             rn);
      if (MODE != 0) ldKz<K, S, T>(fp + sz, inb && more, fn);
    } else {
      if (RAWC) {
        const bool okn = inb && z + 1 < g.nz;
        ldKz<K, S, T>(up + sz, okn, un);
        wn = okn ? dw[(int64_t)(z + 1) * plane + icol] : cx<T>{};
      } else {
        ld_u<K, S, SC, T, PRO, LDSC>(up + sz, inb && z + 1 < g.nz, x, y, z + 1, ec, gc, dw,
                                     (int64_t)(z + 1) * plane + icol, c, un, lc);
      }
      ld_u<K, S, SC, T, PRO, LDSC>(rpp, rin, rx, ry, z, ec, gc, dw, (int64_t)z * plane + rcol, c, rc, lc);
      // the coarse plane the next step adds (the upper parent of z + 2) goes
      // to the slot no plane of this step uses; the barrier below orders it
      if (LDSC && (z & 1) == 0) load_stage((z + 2) / 2);
    }
    if (LDSC && (z & 1) == 0) put_stage();
    if (ring) {
#pragma unroll
      for (int k = 0; k < K; ++k) sm[ro + k] = cx<LE>{(LE)rc[k].re, (LE)rc[k].im};
    }
    // the own point's u at z (RAWC: formed from f, where it is used)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const cx<T> v = RAWC ? wc * uc[k] : uc[k];
      nb[RYS + k] = cx<LE>{(LE)v.re, (LE)v.im};
    }
    if (EF && inb) {
      const int64_t ir = (int64_t)z * plane + icol;
      ldK<K, S, T>(f + ir * g.P + c, fc);
      de = dg[ir];
      if (MODE == 2) we = dw[ir];
    }
    __syncthreads();
    if (inb) {
      const int64_t ir = (int64_t)z * plane + icol;
      const cx<T> d = EF || EF2 ? de : dg[ir];
      cx<T> acc[K], sum[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const cx<T> us = RAWC ? wc * uc[k] : uc[k];
        const cx<T> zp = RAWC ? wn * un[k] : un[k];
        acc[k] = d * us;
        sum[k] = ihz * (um[k] + zp) + ihy * (wid<T>(nb[k]) + wid<T>(nb[2 * RYS + k]));
        sum[k] = sum[k] + ihx * wid<T>(nb[RYS - RX + k]);
        sum[k] = sum[k] + ihx * wid<T>(nb[RYS + RX + k]);
        acc[k] = acc[k] - sum[k];
      }
      const int64_t o = ir * g.P + c;
      if (MODE == 0) {
        stK<K, S, T>(out + o, acc);
      } else {
        // f: RAWC holds it, EF has issued it, PF prefetched it; else now
        if (RAWC) {
#pragma unroll
          for (int k = 0; k < K; ++k) fc[k] = uc[k];
        } else if (!PF && !EF && !EF2) {
          ldK<K, S, T>(f + o, fc);
        }
        cx<T> res[K];
        if (MODE == 1) {
#pragma unroll
          for (int k = 0; k < K; ++k) res[k] = fc[k] - acc[k];
        } else {
          const cx<T> w = RAWC ? wc : (EF || EF2 ? we : dw[ir]);
#pragma unroll
          for (int k = 0; k < K; ++k) res[k] = (RAWC ? wc * uc[k] : uc[k]) + w * (fc[k] - acc[k]);
        }
        stK<K, S, T>(out + o, res);
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      um[k] = RAWC ? wc * uc[k] : uc[k];
      uc[k] = un[k];
      if (PF) {
        un[k] = unn[k];
        rc[k] = rn[k];
        fc[k] = fn[k];
      }
    }
    if (RAWC) wc = wn;
  }
}

template <class S, class T, int MODE, int TY, class SC = S, int PRO = 0>
static void fine_t16_launch(const Geo& g, const void* u, const void* f, void* out, const void* dg, const void* dw,
                            const double ih[3], int zc, hipStream_t s, const void* ec = nullptr,
                            const Geo& gc = Geo{}) {
  constexpr int CG = 128 / (int)sizeof(S);
  ZTiles zt;
  zt.nxb = (g.nx + TB - 1) / TB;
  const int nyb = (g.ny + TY - 1) / TY;
  zt.zc = zc;
  zt.nzc = (g.nz + zt.zc - 1) / zt.zc;
  zt.ntiles = (int64_t)zt.nxb * nyb * zt.nzc * (g.P / CG);
  zt.per = (int)((zt.ntiles + 7) / 8);
  hipLaunchKernelGGL((k_fine_t16<S, T, MODE, TY, SC, PRO>), dim3((unsigned)(8 * (int64_t)zt.per)),
                     dim3(64 * TY), 0, s, g, zt, nyb, (const S*)u, (const S*)f, (S*)out, (const cx<T>*)dg,
                     (const cx<T>*)dw,
                     (T)ih[0], (T)ih[1], (T)ih[2], (const SC*)ec, gc);
}

// ---------------------------------------------------------------------------
// Fused finest-level residual + full-weighting restriction (3D): a 512-lane
// workgroup owns an 8 x 8 tile of coarse nodes for one 64-byte group of
// right-hand sides and a chunk of RZC coarse planes. Marching through the fine
// planes it stages u (with a one-point ring) in LDS, computes the residual on
// the 17 x 17 fine points the tile's nodes need (same operation order as the
// stand-alone residual kernels), stages that residual plane in LDS and adds
// its weighted terms to the coarse nodes' accumulators. A coarse node receives
// its 27 terms in the order of k_restrict (dz outer, then dy, then dx), so
// the result is bitwise that of the residual kernel followed by k_restrict,
// without writing and re-reading the fine residual.
// ---------------------------------------------------------------------------
// Store exactly the K values a lane owns: BF16 pairs are 4 per 16 B, so two
// values (K = 2) go out as one 8-byte store with the same rounding as st16.
template <int K, class SO, class T> __device__ inline void st_own(SO* p, const cx<T>* o) {
  if constexpr (std::is_same<SO, cbf>::value && K == 2) {
    const uint32_t w0 = (uint32_t)f2bf((float)o[0].re) | ((uint32_t)f2bf((float)o[0].im) << 16);
    const uint32_t w1 = (uint32_t)f2bf((float)o[1].re) | ((uint32_t)f2bf((float)o[1].im) << 16);
    *reinterpret_cast<uint2*>(p) = uint2{w0, w1};
  } else {
    static_assert(K % St<SO>::R == 0, "a lane must own whole 16-byte units of the output");
    stK<K, SO, T>(p, o);
  }
}

constexpr int RT = 8;           // coarse tile edge
constexpr int RF = 2 * RT + 1;  // fine residual points per axis
constexpr int RU = RF + 2;      // fine u points per axis (with the ring)
constexpr int RZC = 32;         // coarse planes per z-chunk

template <class S, class SO, class T>
__global__ __launch_bounds__(512) void k_resid_restrict(Geo gf, Geo gc, int ncg, int nxb, int nyb, int64_t ntiles,
                                                        int per, const S* __restrict__ u, const S* __restrict__ f,
                                                        SO* __restrict__ rc, const cx<T>* __restrict__ dg, T ihx,
                                                        T ihy, T ihz) {
  constexpr int CG = 64 / (int)sizeof(S);  // columns per group
  constexpr int K = CG / 4;                 // columns per lane (16 B)
  constexpr int NRES = RF * RF * 4;         // residual tasks (point, slot)
  constexpr int NT = (NRES + 511) / 512;    // residual tasks per lane
  constexpr int NRING = 4 * RU - 4;         // ring points of the u plane
  __shared__ cx<T> su[RU * RU * CG];
  __shared__ cx<T> sr[RF * RF * CG];
  const int64_t t0 = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (t0 >= ntiles) return;  // whole workgroup leaves together
  int64_t t = t0;
  const int cgi = (int)(t % ncg);
  t /= ncg;
  const int yb = (int)(t % nyb);
  t /= nyb;
  const int xb = (int)(t % nxb);
  const int zci = (int)(t / nxb);
  const int Z0 = zci * RZC, Z1 = Z0 + RZC < gc.nz ? Z0 + RZC : gc.nz;
  const int fx0 = 2 * RT * xb, fy0 = 2 * RT * yb;  // fine origin of the residual region
  const int sl = threadIdx.x & 3;                  // the same slot for all of a lane's tasks
  const int c = cgi * CG + sl * K;
  const int64_t plane = (int64_t)gf.nx * gf.ny, sz = plane * gf.P;
  // residual tasks of this lane
  int rx[NT], ry[NT];
  bool rin[NT];
  int64_t rcol[NT];
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    const int task = threadIdx.x + 512 * i;
    const int p = task >> 2;
    rx[i] = p % RF;
    ry[i] = p / RF;
    const int gx = fx0 + rx[i], gy = fy0 + ry[i];
    rin[i] = task < NRES && gx < gf.nx && gy < gf.ny;
    rcol[i] = (int64_t)gy * gf.nx + gx;
  }
  // ring task of this lane (lanes 0 .. 4*NRING-1): u-plane coordinates (hx, hy)
  const int rp = threadIdx.x >> 2;
  int hx, hy;
  if (rp < RU) {
    hx = rp;
    hy = 0;
  } else if (rp < 2 * RU) {
    hx = rp - RU;
    hy = RU - 1;
  } else if (rp < 2 * RU + RF) {
    hx = 0;
    hy = rp - 2 * RU + 1;
  } else {
    hx = RU - 1;
    hy = rp - 2 * RU - RF + 1;
  }
  const bool ring = rp < NRING;
  const int gxr = fx0 + hx - 1, gyr = fy0 + hy - 1;
  const bool ringin = ring && gxr >= 0 && gxr < gf.nx && gyr >= 0 && gyr < gf.ny;
  const int64_t ringcol = (int64_t)gyr * gf.nx + gxr;
  // accumulation task (lanes 0..255): coarse node (ax, ay) of the tile
  const int aq = threadIdx.x >> 2;
  const int ax = aq % RT, ay = aq / RT;
  const int X = RT * xb + ax, Y = RT * yb + ay;
  const bool acc_on = threadIdx.x < 4 * RT * RT && X < gc.nx && Y < gc.ny;
  cx<T> um[NT][K], uc[NT][K], un[NT][K], v[K];
  const int zf0 = 2 * Z0, zf1 = 2 * Z1;  // fine planes of this chunk (inclusive)
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    const S* up = u + ((int64_t)zf0 * plane + rcol[i]) * gf.P + c;
    ldKz<K, S, T>(up - sz, rin[i] && zf0 > 0, um[i]);
    ldKz<K, S, T>(up, rin[i], uc[i]);
  }
  cx<T> accA[K], accB[K];
#pragma unroll
  for (int k = 0; k < K; ++k) accA[k] = accB[k] = {(T)0, (T)0};
  for (int zf = zf0; zf <= zf1; ++zf) {
#pragma unroll
    for (int i = 0; i < NT; ++i)
      ldKz<K, S, T>(u + ((int64_t)(zf + 1) * plane + rcol[i]) * gf.P + c, rin[i] && zf + 1 < gf.nz, un[i]);
    if (ring) {
      ldKz<K, S, T>(u + ((int64_t)zf * plane + ringcol) * gf.P + c, ringin, v);
      const int o = (hy * RU + hx) * CG + sl * K;
#pragma unroll
      for (int k = 0; k < K; ++k) su[o + k] = v[k];
    }
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      if (threadIdx.x + 512 * i >= NRES) continue;
      const int o = ((ry[i] + 1) * RU + rx[i] + 1) * CG + sl * K;
#pragma unroll
      for (int k = 0; k < K; ++k) su[o + k] = uc[i][k];
    }
    // f and D of the plane are issued before the barrier, so that their
    // latency overlaps it (as in the LDS-tiled sweeps)
    cx<T> fv[NT][K], dv[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      if (threadIdx.x + 512 * i >= NRES || !rin[i]) continue;
      const int64_t ir = (int64_t)zf * plane + rcol[i];
      dv[i] = dg[ir];
      ldK<K, S, T>(f + ir * gf.P + c, fv[i]);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      if (threadIdx.x + 512 * i >= NRES) continue;
      cx<T> res[K];
      if (rin[i]) {
        const int o = ((ry[i] + 1) * RU + rx[i] + 1) * CG + sl * K;
        const cx<T> d = dv[i];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          cx<T> acc = d * uc[i][k];
          cx<T> sum = ihz * (um[i][k] + un[i][k]) + ihy * (su[o - RU * CG + k] + su[o + RU * CG + k]);
          sum = sum + ihx * su[o - CG + k];
          sum = sum + ihx * su[o + CG + k];
          acc = acc - sum;
          res[k] = fv[i][k] - acc;
        }
      } else {
#pragma unroll
        for (int k = 0; k < K; ++k) res[k] = {(T)0, (T)0};
      }
      const int orr = (ry[i] * RF + rx[i]) * CG + sl * K;
#pragma unroll
      for (int k = 0; k < K; ++k) sr[orr + k] = res[k];
    }
    __syncthreads();
    if (acc_on) {
      // fine plane zf = 2 Z + 1 + dz: odd planes are dz = 0 of Z = (zf - 1) / 2;
      // even planes close Z = zf / 2 - 1 (dz = +1) and open Z = zf / 2 (dz = -1)
      const bool odd = zf & 1;
      const int nrole = odd ? 1 : 2;
      for (int role = 0; role < nrole; ++role) {
        const int dz = odd ? 0 : (role == 0 ? 1 : -1);
        const int Zc = odd ? (zf - 1) / 2 : (role == 0 ? zf / 2 - 1 : zf / 2);
        if (Zc < Z0 || Zc >= Z1) continue;
        cx<T>* acc = role == 0 ? accA : accB;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
          for (int dx = -1; dx <= 1; ++dx) {
            const T w = (dx ? (T)0.5 : (T)1) * (dy ? (T)0.5 : (T)1) * (dz ? (T)0.5 : (T)1);
            const int o = ((2 * ay + 1 + dy) * RF + 2 * ax + 1 + dx) * CG + sl * K;
#pragma unroll
            for (int k = 0; k < K; ++k) acc[k] = acc[k] + w * sr[o + k];
          }
        if (dz == 1) {  // Zc complete
          cx<T> outv[K];
#pragma unroll
          for (int k = 0; k < K; ++k) outv[k] = (T)0.125 * accA[k];
          const int64_t I = ((int64_t)Zc * gc.ny + Y) * gc.nx + X;
          st_own<K, SO, T>(rc + I * gc.P + c, outv);
        }
      }
      if (!odd) {  // the plane opened on accB continues on accA
#pragma unroll
        for (int k = 0; k < K; ++k) {
          accA[k] = accB[k];
          accB[k] = {(T)0, (T)0};
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        um[i][k] = uc[i][k];
        uc[i][k] = un[i][k];
      }
  }
}

template <class S, class SO, class T>
static void resid_restrict_launch(const Geo& gf, const Geo& gc, const void* u, const void* f, void* rc, const void* dg,
                                  const double ih[3], hipStream_t s) {
  constexpr int CG = 64 / (int)sizeof(S);
  const int ncg = gf.P / CG;
  const int nxb = (gc.nx + RT - 1) / RT, nyb = (gc.ny + RT - 1) / RT, nzc = (gc.nz + RZC - 1) / RZC;
  const int64_t ntiles = (int64_t)ncg * nxb * nyb * nzc;
  const int per = (int)((ntiles + 7) / 8);
  hipLaunchKernelGGL((k_resid_restrict<S, SO, T>), dim3((unsigned)(8 * (int64_t)per)), dim3(512), 0, s, gf, gc, ncg, nxb,
                     nyb, ntiles, per, (const S*)u, (const S*)f, (SO*)rc, (const cx<T>*)dg, (T)ih[0], (T)ih[1],
                     (T)ih[2]);
}

// ---------------------------------------------------------------------------
// Fused pre-smoothing, residual and restriction on the finest 3D level (the
// cycle with two pre-sweeps): from f alone, u1 = (w/D) f (the sweep from a
// zero guess), u2 = u1 + (w/D)(f - M u1) (the second sweep), then
// r = f - M u2 and r_c = R r, in one pass. The tile is that of
// k_resid_restrict (8 x 8 coarse nodes, one 64-byte column group, a chunk of
// RZC coarse planes): the residual needs u2 on the 19 x 19 points around its
// 17 x 17 fine points, and u2 there needs u1 on 21 x 21. Marching through the
// fine planes t, a workgroup forms u1(t) (LDS, with its ring), then u2(t) on
// 19 x 19 (kept one plane in LDS for the residual's in-plane neighbours),
// writes the u2 points the tile owns, and forms the residual of plane t - 1,
// which the restriction of k_resid_restrict takes up one plane later. Every
// value is formed with the operations, and in the order, of the sweep
// kernels and of k_resid_restrict, so u2 and r_c are bitwise those of the
// unfused path; u2 is written but never re-read, and f is read once. Each
// LDS plane is double-buffered, so one barrier per plane suffices, and every
// global load is issued one plane ahead of its use.
// ---------------------------------------------------------------------------
constexpr int RV = RU + 2;  // fine u1 points per axis (the ring of the u2 region)
// Lanes per workgroup: 768 for FP32 fields (two u2 tasks per lane, about 140
// VGPRs with the next plane's loads in flight; 1024 lanes, at 128 VGPRs,
// spilled); FP64 fields need more registers per task and run 512 lanes.
template <class T> constexpr int prr_lanes() { return sizeof(T) == 4 ? 768 : 512; }

template <class S, class SO, class T, int PRR_L = prr_lanes<T>()>
__global__ __launch_bounds__(PRR_L) void k_pre_rr(Geo gf, Geo gc, int ncg, int nxb, int nyb, int64_t ntiles, int per,
                                                const S* __restrict__ f, S* __restrict__ u2o, SO* __restrict__ rc,
                                                const cx<T>* __restrict__ dg, const cx<T>* __restrict__ dw, T ihx,
                                                T ihy, T ihz) {
  constexpr int CG = 64 / (int)sizeof(S);  // columns per group
  constexpr int K = CG / 4;                 // columns per lane (16 B)
  constexpr int NU = RU * RU * 4;           // u2 tasks (point, slot)
  constexpr int NT = (NU + PRR_L - 1) / PRR_L;  // u2 tasks per lane
  constexpr int NRV = 4 * RV - 4;           // ring points of the u1 region
  // plane rings: u1 of t (and t - 1, the z - 1 neighbour of u2(t)), u2 of
  // t - 1 (and t - 2, the z - 1 neighbour of r(t - 1)), by plane parity
  __shared__ cx<T> sv2[2][RV * RV * CG];  // u1, with the ring
  __shared__ cx<T> su2[2][RU * RU * CG];  // u2
  __shared__ cx<T> sr2[2][RF * RF * CG];  // r(t - 1) (and r(t - 2), restricted one plane later)
  const int64_t t0 = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (t0 >= ntiles) return;  // whole workgroup leaves together
  int64_t tt = t0;
  const int cgi = (int)(tt % ncg);
  tt /= ncg;
  const int yb = (int)(tt % nyb);
  tt /= nyb;
  const int xb = (int)(tt % nxb);
  const int zci = (int)(tt / nxb);
  const int Z0 = zci * RZC, Z1 = Z0 + RZC < gc.nz ? Z0 + RZC : gc.nz;
  const bool last_chunk = Z1 == gc.nz;
  const int fx0 = 2 * RT * xb, fy0 = 2 * RT * yb;  // fine origin of the residual region
  const int sl = threadIdx.x & 3;                  // the same slot for all of a lane's tasks
  const int c = cgi * CG + sl * K;
  const int64_t plane = (int64_t)gf.nx * gf.ny;
  // Addresses split into a plane part, the same for the whole workgroup (held
  // in scalar registers), and a lane part fixed for the whole march: the
  // element offsets of the lane's columns within a plane
  const int64_t planeP = plane * gf.P, cplaneP = (int64_t)gc.nx * gc.ny * gc.P;
  // u2 tasks of this lane: point (ux, uy) of the 19 x 19 region (fine
  // (fx0 - 1 + ux, fy0 - 1 + uy)); the inner 17 x 17 are residual points
  int ux[NT], uy[NT];
  bool uon[NT], uin[NT], res[NT], own[NT];
  int64_t ucol[NT], ucolP[NT];
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    const int task = threadIdx.x + PRR_L * i;
    const int p = task >> 2;
    uon[i] = task < NU;
    ux[i] = p % RU;
    uy[i] = p / RU;
    const int gx = fx0 - 1 + ux[i], gy = fy0 - 1 + uy[i];
    uin[i] = uon[i] && gx >= 0 && gx < gf.nx && gy >= 0 && gy < gf.ny;
    res[i] = uon[i] && ux[i] >= 1 && ux[i] <= RF && uy[i] >= 1 && uy[i] <= RF;
    // the u2 points this tile writes: its 16 x 16 core (every fine point once)
    own[i] = uin[i] && ux[i] >= 1 && ux[i] <= 2 * RT && uy[i] >= 1 && uy[i] <= 2 * RT;
    ucol[i] = uin[i] ? (int64_t)gy * gf.nx + gx : 0;
    ucolP[i] = ucol[i] * gf.P + c;
  }
  // ring task of this lane (lanes 0 .. 4*NRV-1): u1-region coordinates (hx, hy)
  const int rp = threadIdx.x >> 2;
  int hx, hy;
  if (rp < RV) {
    hx = rp;
    hy = 0;
  } else if (rp < 2 * RV) {
    hx = rp - RV;
    hy = RV - 1;
  } else if (rp < 2 * RV + RU) {
    hx = 0;
    hy = rp - 2 * RV + 1;
  } else {
    hx = RV - 1;
    hy = rp - 2 * RV - RU + 1;
  }
  const bool ring = rp < NRV;
  const int gxr = fx0 - 2 + hx, gyr = fy0 - 2 + hy;
  const bool ringin = ring && gxr >= 0 && gxr < gf.nx && gyr >= 0 && gyr < gf.ny;
  const int64_t ringcol = ringin ? (int64_t)gyr * gf.nx + gxr : 0;
  const int64_t ringcolP = ringcol * gf.P + c;
  // accumulation task (lanes 0..255): coarse node (ax, ay) of the tile
  const int aq = threadIdx.x >> 2;
  const int ax = aq % RT, ay = aq / RT;
  const int X = RT * xb + ax, Y = RT * yb + ay;
  const bool acc_on = threadIdx.x < 4 * RT * RT && X < gc.nx && Y < gc.ny;
  const int64_t xyP = ((int64_t)Y * gc.nx + X) * gc.P + c;
  // per task: f at t - 1 (residual), t, t + 1; w/D at t, t + 1; D at t - 1
  // (residual) and t; the ring's f and w/D at t
  cx<T> fR[NT][K], fA[NT][K], fB[NT][K];
  cx<T> wA[NT], wB[NT], dA[NT], dR[NT];
  cx<T> frA[K], wrA{};
  const int zf0 = 2 * Z0, zf1 = 2 * Z1;  // residual planes of this chunk (inclusive)
  const int tb = zf0 - 1, te = zf1 + 1;  // u2 planes this chunk forms
  auto ok_plane = [&](int z) { return z >= 0 && z < gf.nz; };
  // Every global load is issued by every lane, from a clamped address, and
  // zeroed where it lies outside the grid or the lane has no such task: with
  // no load behind a branch, a wait for one plane's operands leaves the next
  // plane's loads in flight.
  auto ld_f = [&](int z, int64_t colP, bool ok, cx<T>* o) {
    const int zc = z < 0 ? 0 : (z >= gf.nz ? gf.nz - 1 : z);
    ldK<K, S, T>(f + (int64_t)zc * planeP + colP, o);
#pragma unroll
    for (int k = 0; k < K; ++k) o[k] = ok ? o[k] : cx<T>{};
  };
  auto ld_c = [&](const cx<T>* a, int z, int64_t col, bool ok) {
    const int zc = z < 0 ? 0 : (z >= gf.nz ? gf.nz - 1 : z);
    const cx<T> v = a[(int64_t)zc * plane + col];
    return ok ? v : cx<T>{};
  };
  // prologue: u1(tb - 1) of the own points into its plane slot (only the own
  // point of it is read); f and w/D of planes tb and tb + 1, D and the ring of
  // plane tb
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    const bool okm = uin[i] && ok_plane(tb - 1), okc = uin[i] && ok_plane(tb), okn = uin[i] && ok_plane(tb + 1);
    cx<T> fm[K];
    ld_f(tb - 1, ucolP[i], okm, fm);
    const cx<T> wm = ld_c(dw, tb - 1, ucol[i], okm);
    if (uon[i]) {
      const int o = ((uy[i] + 1) * RV + ux[i] + 1) * CG + sl * K;
#pragma unroll
      for (int k = 0; k < K; ++k) sv2[(tb - 1) & 1][o + k] = wm * fm[k];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) fR[i][k] = cx<T>{};
    ld_f(tb, ucolP[i], okc, fA[i]);
    wA[i] = ld_c(dw, tb, ucol[i], okc);
    ld_f(tb + 1, ucolP[i], okn, fB[i]);
    wB[i] = ld_c(dw, tb + 1, ucol[i], okn);
    dA[i] = ld_c(dg, tb, ucol[i], okc);
    dR[i] = cx<T>{};
  }
  {
    const bool ok = ringin && ok_plane(tb);
    ld_f(tb, ringcolP, ok, frA);
    wrA = ld_c(dw, tb, ringcol, ok);
  }
  cx<T> accA[K], accB[K];
#pragma unroll
  for (int k = 0; k < K; ++k) accA[k] = accB[k] = {(T)0, (T)0};
  // the restriction of residual plane zf (sr: that plane), as k_resid_restrict
  // adds it
  auto restrict_plane = [&](int zf, const cx<T>* sr) {
    if (zf < zf0 || zf > zf1 || !acc_on) return;
    // fine plane zf = 2 Z + 1 + dz: odd planes are dz = 0 of Z = (zf - 1) / 2;
    // even planes close Z = zf / 2 - 1 (dz = +1) and open Z = zf / 2 (dz = -1)
    const bool odd = zf & 1;
    const int nrole = odd ? 1 : 2;
    for (int role = 0; role < nrole; ++role) {
      const int dz = odd ? 0 : (role == 0 ? 1 : -1);
      const int Zc = odd ? (zf - 1) / 2 : (role == 0 ? zf / 2 - 1 : zf / 2);
      if (Zc < Z0 || Zc >= Z1) continue;
      cx<T>* acc = role == 0 ? accA : accB;
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const T w = (dx ? (T)0.5 : (T)1) * (dy ? (T)0.5 : (T)1) * (dz ? (T)0.5 : (T)1);
          const int o = ((2 * ay + 1 + dy) * RF + 2 * ax + 1 + dx) * CG + sl * K;
#pragma unroll
          for (int k = 0; k < K; ++k) acc[k] = acc[k] + w * sr[o + k];
        }
      if (dz == 1) {  // Zc complete
        cx<T> outv[K];
#pragma unroll
        for (int k = 0; k < K; ++k) outv[k] = (T)0.125 * accA[k];
        st_own<K, SO, T>(rc + (int64_t)Zc * cplaneP + xyP, outv);
      }
    }
    if (!odd) {  // the plane opened on accB continues on accA
#pragma unroll
      for (int k = 0; k < K; ++k) {
        accA[k] = accB[k];
        accB[k] = {(T)0, (T)0};
      }
    }
  };
  // One barrier per plane: after it, every lane's u1(t) and ring are in LDS,
  // and so are u2(t - 1) and the residual of plane t - 2 (written during the
  // previous plane), which is restricted first. Each buffer alternates by
  // plane parity, so what one plane writes is read after the next barrier.
  // Every global load is issued one plane before its use and stays in flight
  // across the barrier, which waits for the workgroup's LDS operations only.
  for (int t = tb; t <= te; ++t) {
    cx<T>* const sv = sv2[t & 1];        // u1(t)
    const cx<T>* const svm = sv2[(t - 1) & 1];  // u1(t - 1)
    cx<T>* const su = su2[(t - 1) & 1];  // u2(t - 1); u2(t) goes to the other slot
    const cx<T>* const sum2 = su2[t & 1];  // u2(t - 2)
    // u1(t) into LDS: own points and the ring (the sweep from zero, w/D f)
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      if (!uon[i]) continue;
      const int o = ((uy[i] + 1) * RV + ux[i] + 1) * CG + sl * K;
#pragma unroll
      for (int k = 0; k < K; ++k) sv[o + k] = wA[i] * fA[i][k];
    }
    if (ring) {
      const int o = (hy * RV + hx) * CG + sl * K;
#pragma unroll
      for (int k = 0; k < K; ++k) sv[o + k] = wrA * frA[k];
    }
    // the loads of the next plane: its ring and D, f and w/D of plane t + 2
    cx<T> frB[K], wrB{};
    {
      const bool ok = ringin && ok_plane(t + 1);
      ld_f(t + 1, ringcolP, ok, frB);
      wrB = ld_c(dw, t + 1, ringcol, ok);
    }
    cx<T> fC[NT][K], wC[NT], dB[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      const bool okn = uin[i] && ok_plane(t + 1), ok2 = uin[i] && ok_plane(t + 2);
      dB[i] = ld_c(dg, t + 1, ucol[i], okn);
      ld_f(t + 2, ucolP[i], ok2, fC[i]);
      wC[i] = ld_c(dw, t + 2, ucol[i], ok2);
    }
    __syncthreads();
    restrict_plane(t - 2, sr2[(t - 1) & 1]);
    // u2(t) on the 19 x 19 region: the second sweep, as the LDS-tiled sweep
    // forms it (0 outside the grid)
    const bool tin = ok_plane(t);
    const bool t_own = t >= zf0 && (t < zf1 || (last_chunk && t == zf1)) && tin;
    cx<T> u2c[NT][K];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
#pragma unroll
      for (int k = 0; k < K; ++k) u2c[i][k] = cx<T>{};
      if (!uin[i] || !tin) continue;
      const int o = ((uy[i] + 1) * RV + ux[i] + 1) * CG + sl * K;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const cx<T> us = wA[i] * fA[i][k];
        const cx<T> zp = wB[i] * fB[i][k];
        cx<T> acc = dA[i] * us;
        cx<T> sum = ihz * (svm[o + k] + zp) + ihy * (sv[o - RV * CG + k] + sv[o + RV * CG + k]);
        sum = sum + ihx * sv[o - CG + k];
        sum = sum + ihx * sv[o + CG + k];
        acc = acc - sum;
        u2c[i][k] = us + wA[i] * (fA[i][k] - acc);
      }
      if (own[i] && t_own) stK<K, S, T>(u2o + (int64_t)t * planeP + ucolP[i], u2c[i]);
    }
    // the residual of plane t - 1 (u2 of t - 1 in LDS, of t - 2 and t in
    // registers), as k_resid_restrict forms it, into sr
    const int zr = t - 1;
    const bool do_res = zr >= zf0 && zr <= zf1;
    if (do_res) {
#pragma unroll
      for (int i = 0; i < NT; ++i) {
        if (!res[i]) continue;
        cx<T> rv[K];
        if (uin[i]) {
          const int o = (uy[i] * RU + ux[i]) * CG + sl * K;
          const cx<T> d = dR[i];
#pragma unroll
          for (int k = 0; k < K; ++k) {
            cx<T> acc = d * su[o + k];
            cx<T> sum = ihz * (sum2[o + k] + u2c[i][k]) + ihy * (su[o - RU * CG + k] + su[o + RU * CG + k]);
            sum = sum + ihx * su[o - CG + k];
            sum = sum + ihx * su[o + CG + k];
            acc = acc - sum;
            rv[k] = fR[i][k] - acc;
          }
        } else {
#pragma unroll
          for (int k = 0; k < K; ++k) rv[k] = {(T)0, (T)0};
        }
        const int orr = ((uy[i] - 1) * RF + ux[i] - 1) * CG + sl * K;
#pragma unroll
        for (int k = 0; k < K; ++k) sr2[t & 1][orr + k] = rv[k];
      }
    }
    // u2(t) into the slot of u2(t - 2) (its only reader in this plane is this
    // lane's own residual above; the neighbours of u2(t - 2) were read before
    // this plane's barrier); shift the planes
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      if (uon[i]) {
        const int o = (uy[i] * RU + ux[i]) * CG + sl * K;
#pragma unroll
        for (int k = 0; k < K; ++k) su2[t & 1][o + k] = u2c[i][k];
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        fR[i][k] = fA[i][k];
        fA[i][k] = fB[i][k];
        fB[i][k] = fC[i][k];
      }
      dR[i] = dA[i];
      dA[i] = dB[i];
      wA[i] = wB[i];
      wB[i] = wC[i];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) frA[k] = frB[k];
    wrA = wrB;
  }
  // the residual of the last plane, written before the loop ended
  __syncthreads();
  restrict_plane(te - 1, sr2[te & 1]);
}

template <class S, class SO, class T>
static void pre_rr_launch(const Geo& gf, const Geo& gc, const void* f, void* u2, void* rc, const void* dg,
                          const void* dw, const double ih[3], hipStream_t s) {
  constexpr int CG = 64 / (int)sizeof(S);
  const int ncg = gf.P / CG;
  const int nxb = (gc.nx + RT - 1) / RT, nyb = (gc.ny + RT - 1) / RT, nzc = (gc.nz + RZC - 1) / RZC;
  const int64_t ntiles = (int64_t)ncg * nxb * nyb * nzc;
  const int per = (int)((ntiles + 7) / 8);
  hipLaunchKernelGGL((k_pre_rr<S, SO, T>), dim3((unsigned)(8 * (int64_t)per)), dim3(prr_lanes<T>()), 0, s, gf, gc,
                     ncg, nxb, nyb,
                     ntiles, per, (const S*)f, (S*)u2, (SO*)rc, (const cx<T>*)dg, (const cx<T>*)dw, (T)ih[0],
                     (T)ih[1], (T)ih[2]);
}

// ---------------------------------------------------------------------------
// 3D Galerkin-level operator (27-point stencil), z-marching through LDS: a
// 256-lane workgroup owns an 8 x 8 tile of grid columns for one 128-byte group
// of right-hand sides (32 BF16 pairs, 16 complex64 or 8 complex128) and a
// chunk of z planes. The planes z-1, z, z+1 of the tile with its one-point
// ring sit in a three-plane LDS ring in storage precision; each step loads
// only plane z+2's tile. The 27 products are accumulated in the order of
// k_gal, so results are bitwise those of k_gal. Modes APPLY, RESID, JAC.
// ---------------------------------------------------------------------------
constexpr int GT = 8;            // tile edge
constexpr int GH = GT + 2;       // with the ring
constexpr int GZC = 16;          // planes per chunk (fewer on small grids)

template <class S, class T, int MODE>
__global__ __launch_bounds__(256) void k_gal_lds(Geo g, int ncg, int nxb, int nyb, int zc, int64_t ntiles, int per,
                                                 const S* __restrict__ u, const S* __restrict__ f,
                                                 S* __restrict__ out, const cx<T>* __restrict__ st,
                                                 const cx<T>* __restrict__ dw) {
  constexpr int CB = 128;                          // bytes per point and group
  constexpr int CG = CB / (int)sizeof(S);          // columns per group
  constexpr int K = CG / 4;                        // columns per lane
  constexpr int U16 = CB / 16;                     // 16-byte units per point and group
  constexpr int R = St<S>::R;                      // columns per 16-byte unit
  __shared__ uint4 sp[3][GH * GH * U16];
  const int64_t t0 = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (t0 >= ntiles) return;  // whole workgroup leaves together
  int64_t t = t0;
  const int cgi = (int)(t % ncg);
  t /= ncg;
  const int yb = (int)(t % nyb);
  t /= nyb;
  const int xb = (int)(t % nxb);
  const int zci = (int)(t / nxb);
  const int z0 = zci * zc, z1 = z0 + zc < g.nz ? z0 + zc : g.nz;
  const int q = threadIdx.x >> 2, sl = threadIdx.x & 3;
  const int px = q % GT, py = q / GT;
  const int x = xb * GT + px, y = yb * GT + py;
  const bool inb = x < g.nx && y < g.ny;
  const int c = cgi * CG + sl * K;
  const int64_t plane = (int64_t)g.nx * g.ny;
  // loads one plane's tile (with the ring) into LDS buffer b; zero outside the grid
  auto load_plane = [&](int zz, int b) {
    for (int e = threadIdx.x; e < GH * GH * U16; e += 256) {
      const int hp = e / U16, w = e - hp * U16;
      const int gx = xb * GT + hp % GH - 1, gy = yb * GT + hp / GH - 1;
      uint4 val{0u, 0u, 0u, 0u};
      if (zz >= 0 && zz < g.nz && gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny)
        val = *reinterpret_cast<const uint4*>(u + ((int64_t)zz * plane + (int64_t)gy * g.nx + gx) * g.P + cgi * CG +
                                              w * R);
      sp[b][e] = val;
    }
  };
  load_plane(z0 - 1, (z0 + 2) % 3);
  load_plane(z0, z0 % 3);
  const int me = ((py + 1) * GH + px + 1) * U16 + sl * (K / R);
  for (int z = z0; z < z1; ++z) {
    load_plane(z + 1, (z + 1) % 3);
    __syncthreads();
    if (inb) {
      const int64_t i = (int64_t)z * plane + (int64_t)y * g.nx + x;
      const cx<T>* spn = st + i * 27;
      cx<T> acc[K], nb[K], uc[K];
#pragma unroll
      for (int k = 0; k < K; ++k) acc[k] = {(T)0, (T)0};
#pragma unroll 3
      for (int o = 0; o < 27; ++o) {
        const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
        const uint4* src = &sp[(z + oz + 3) % 3][me + (oy * GH + ox) * U16];
#pragma unroll
        for (int k = 0; k < K; k += R) ld16<T>(reinterpret_cast<const S*>(src + k / R), nb + k);
        if (o == 13) {
#pragma unroll
          for (int k = 0; k < K; ++k) uc[k] = nb[k];
        }
        const cx<T> a = spn[o];
#pragma unroll
        for (int k = 0; k < K; ++k) cfma(acc[k], a, nb[k]);
      }
      const int64_t base = i * g.P + c;
      if (MODE == 0) {
        stK<K, S, T>(out + base, acc);
      } else {
        cx<T> fv[K], res[K];
        ldK<K, S, T>(f + base, fv);
        if (MODE == 1) {
#pragma unroll
          for (int k = 0; k < K; ++k) res[k] = fv[k] - acc[k];
        } else {
          const cx<T> w = dw[i];
#pragma unroll
          for (int k = 0; k < K; ++k) res[k] = uc[k] + w * (fv[k] - acc[k]);
        }
        stK<K, S, T>(out + base, res);
      }
    }
    __syncthreads();
  }
}

template <class S, class T, int MODE>
static bool gal_lds_launch(const Geo& g, const void* u, const void* f, void* out, const void* st, const void* dw,
                           hipStream_t s) {
  constexpr int CG = 128 / (int)sizeof(S);
  if (g.P % CG != 0) return false;
  const int ncg = g.P / CG;
  const int nxb = (g.nx + GT - 1) / GT, nyb = (g.ny + GT - 1) / GT;
  // shorter z-chunks on small grids, so that the launch still has about six
  // workgroups per compute unit (the result does not depend on the chunking)
  int zc = GZC;
  while (zc > 4 && (int64_t)ncg * nxb * nyb * ((g.nz + zc - 1) / zc) < 1536) zc /= 2;
  const int nzc = (g.nz + zc - 1) / zc;
  const int64_t ntiles = (int64_t)ncg * nxb * nyb * nzc;
  const int per = (int)((ntiles + 7) / 8);
  hipLaunchKernelGGL((k_gal_lds<S, T, MODE>), dim3((unsigned)(8 * (int64_t)per)), dim3(256), 0, s, g, ncg, nxb, nyb,
                     zc, ntiles, per, (const S*)u, (const S*)f, (S*)out, (const cx<T>*)st, (const cx<T>*)dw);
  return true;
}

static thread_local FineTile g_tile = {4, 32};
void set_fine_tile(FineTile t) { g_tile = t; }
FineTile get_fine_tile() { return g_tile; }

// The fused finest-level kernels run with the LDS-blocked tiles only (the
// register-blocked family keeps the separate kernels, and the tile-identity
// test compares the two), unless HELM_FUSE=0.
static bool fused_tiles() {
  if (g_tile.ry != 8 && g_tile.ry != 16) return false;
  static const bool off = [] {
    const char* e = std::getenv("HELM_FUSE");
    return e && std::strcmp(e, "0") == 0;
  }();
  return !off;
}

bool can_prolong_sweep(Prec pc, Prec pf, Prec pt, const Geo& gf) {
  return fused_tiles() && ((pf == P32 && pc == PBF && pt == P32 && gf.P % 16 == 0) ||
                           (pf == P64 && pc == P64 && pt == P64 && gf.P % 8 == 0));
}

bool can_resid_restrict(Prec pf, Prec pc, Prec pt, const Geo& gf) {
  return fused_tiles() && ((pf == P32 && (pc == PBF || pc == P32) && pt == P32 && gf.P % 8 == 0) ||
                           (pf == P64 && pc == P64 && pt == P64 && gf.P % 4 == 0));
}

bool launch_prolong_sweep(Prec pc, Prec pf, Prec pt, const Geo& gf, const Geo& gc, const void* ec, const void* u,
                          const void* f, void* out, const void* dg, const void* dw, const double ih[3],
                          hipStream_t s) {
  if (!can_prolong_sweep(pc, pf, pt, gf)) return false;
  const int zc = g_tile.zc > 0 ? g_tile.zc : 32;
  if (pf == P32 && pc == PBF && pt == P32 && gf.P % 16 == 0) {
    if (g_tile.ry == 16)
      fine_t16_launch<c64, float, 2, 16, cbf, 1>(gf, u, f, out, dg, dw, ih, zc, s, ec, gc);
    else
      fine_t16_launch<c64, float, 2, 8, cbf, 1>(gf, u, f, out, dg, dw, ih, zc, s, ec, gc);
    return true;
  }
  if (pf == P64 && pc == P64 && pt == P64 && gf.P % 8 == 0) {
    if (g_tile.ry == 16)
      fine_t16_launch<c128, double, 2, 16, c128, 1>(gf, u, f, out, dg, dw, ih, zc, s, ec, gc);
    else
      fine_t16_launch<c128, double, 2, 8, c128, 1>(gf, u, f, out, dg, dw, ih, zc, s, ec, gc);
    return true;
  }
  return false;
}

bool can_sweep01(Prec pf, Prec pt, const Geo& g) {
  return fused_tiles() && ((pf == P32 && pt == P32 && g.P % 16 == 0) || (pf == P64 && pt == P64 && g.P % 8 == 0));
}

void launch_sweep01(Prec pf, Prec pt, const Geo& g, const void* f, void* out, const void* dg, const void* dw,
                    const double ih[3], hipStream_t s) {
  if (!can_sweep01(pf, pt, g)) fatal_combo("launch_sweep01");
  const int zc = g_tile.zc > 0 ? g_tile.zc : 32;
  // the zero-guess sweep's output is formed on the fly from f (PRO = 2)
  if (pf == P32) {
    if (g_tile.ry == 16)
      fine_t16_launch<c64, float, 2, 16, c64, 2>(g, f, f, out, dg, dw, ih, zc, s);
    else
      fine_t16_launch<c64, float, 2, 8, c64, 2>(g, f, f, out, dg, dw, ih, zc, s);
  } else {
    if (g_tile.ry == 16)
      fine_t16_launch<c128, double, 2, 16, c128, 2>(g, f, f, out, dg, dw, ih, zc, s);
    else
      fine_t16_launch<c128, double, 2, 8, c128, 2>(g, f, f, out, dg, dw, ih, zc, s);
  }
}

bool launch_resid_restrict(Prec pf, Prec pc, Prec pt, const Geo& gf, const Geo& gc, const void* u, const void* f,
                           void* rc, const void* dg, const double ih[3], hipStream_t s) {
  if (!can_resid_restrict(pf, pc, pt, gf)) return false;
  if (pf == P32 && pc == PBF && pt == P32 && gf.P % 8 == 0) {
    resid_restrict_launch<c64, cbf, float>(gf, gc, u, f, rc, dg, ih, s);
    return true;
  }
  if (pf == P32 && pc == P32 && pt == P32 && gf.P % 8 == 0) {
    resid_restrict_launch<c64, c64, float>(gf, gc, u, f, rc, dg, ih, s);
    return true;
  }
  if (pf == P64 && pc == P64 && pt == P64 && gf.P % 4 == 0) {
    resid_restrict_launch<c128, c128, double>(gf, gc, u, f, rc, dg, ih, s);
    return true;
  }
  return false;
}

bool can_pre_rr(Prec pf, Prec pc, Prec pt, const Geo& gf) {
  return can_sweep01(pf, pt, gf) && can_resid_restrict(pf, pc, pt, gf);
}

bool launch_pre_rr(Prec pf, Prec pc, Prec pt, const Geo& gf, const Geo& gc, const void* f, void* u2, void* rc,
                   const void* dg, const void* dw, const double ih[3], hipStream_t s) {
  if (!can_pre_rr(pf, pc, pt, gf)) return false;
  if (pf == P32 && pc == PBF && pt == P32) {
    pre_rr_launch<c64, cbf, float>(gf, gc, f, u2, rc, dg, dw, ih, s);
    return true;
  }
  if (pf == P32 && pc == P32 && pt == P32) {
    pre_rr_launch<c64, c64, float>(gf, gc, f, u2, rc, dg, dw, ih, s);
    return true;
  }
  if (pf == P64 && pc == P64 && pt == P64) {
    pre_rr_launch<c128, c128, double>(gf, gc, f, u2, rc, dg, dw, ih, s);
    return true;
  }
  return false;
}

template <class SU, class SF, class SO, class T, int MODE, int RY>
static void fine_zm_launch(const Geo& g, int L, const void* u, const void* f, void* out, const void* dg,
                           const void* dw, const double ih[3], int zc, hipStream_t s) {
  ZTiles zt;
  const int PPB = 256 / L;
  zt.nxb = (g.nx + PPB - 1) / PPB;
  zt.zc = zc;
  zt.nzc = (g.nz + zt.zc - 1) / zt.zc;
  zt.ntiles = (int64_t)zt.nxb * ((g.ny + RY - 1) / RY) * zt.nzc;
  zt.per = (int)((zt.ntiles + 7) / 8);
  hipLaunchKernelGGL((k_fine_zm<SU, SF, SO, T, MODE, RY>), dim3((unsigned)(8 * (int64_t)zt.per)), dim3(256), 0, s,
                     g, zt, (const SU*)u, (const SF*)f, (SO*)out, (const cx<T>*)dg, (const cx<T>*)dw, (T)ih[0],
                     (T)ih[1], (T)ih[2]);
}

template <class SU, class SF, class SO, class T, int MODE>
static void fine_dispatch(int dim, const Geo& g, const void* u, const void* f, void* out, const void* dg,
                          const void* dw, const double ih[3], hipStream_t s) {
  constexpr int K = kmax3<SU, SF, SO>();
  const int L = g.P / K;
  if (dim == 3 && MODE != 3 && L <= 256) {
    // one row per lane when the output is wider than the input or the
    // arithmetic is FP64 on two values per lane (keeps those outer products
    // at 5-6 waves per SIMD); otherwise the tuned shape
    const int ry = sizeof(SO) > sizeof(SU) || (sizeof(T) == 8 && K >= 2) ? 1 : g_tile.ry;
    const int zc = g_tile.zc > 0 ? g_tile.zc : 32;
    // the LDS-blocked tiles; also for the FP64-arithmetic apply of c64 fields
    // (the outer W = H Z), whose tile stays in storage precision in LDS. The
    // FP64 true residual of c128 fields rounded to a c64 output stays on the
    // register-blocked kernel: at 192^3 x 64 it takes 4.6 ms there and 5.1 ms
    // on the tile (same results bitwise).
    if constexpr (std::is_same<SU, SF>::value && std::is_same<SU, SO>::value &&
                  ((std::is_same<SU, c64>::value && std::is_same<T, float>::value) ||
                   (std::is_same<SU, c128>::value && std::is_same<T, double>::value) ||
                   (std::is_same<SU, c64>::value && std::is_same<T, double>::value && MODE == 0))) {
      const int rt = g_tile.ry;
      if ((rt == 16 || rt == 8) && g.P % (128 / (int)sizeof(SU)) == 0 && MODE != 3) {
        if (rt == 16)
          fine_t16_launch<SU, T, MODE, 16>(g, u, f, out, dg, dw, ih, zc, s);
        else
          fine_t16_launch<SU, T, MODE, 8>(g, u, f, out, dg, dw, ih, zc, s);
        return;
      }
    }
    if (ry == 1)
      fine_zm_launch<SU, SF, SO, T, MODE, 1>(g, L, u, f, out, dg, dw, ih, zc, s);
    else if (ry == 2)
      fine_zm_launch<SU, SF, SO, T, MODE, 2>(g, L, u, f, out, dg, dw, ih, zc, s);
    else
      fine_zm_launch<SU, SF, SO, T, MODE, 4>(g, L, u, f, out, dg, dw, ih, zc, s);
    return;
  }
  const int64_t thr = g.npts * (g.P / K);
  if (dim == 3)
    hipLaunchKernelGGL((k_fine<3, SU, SF, SO, T, MODE>), grid1(thr), dim3(256), 0, s, g, (const SU*)u, (const SF*)f,
                       (SO*)out, (const cx<T>*)dg, (const cx<T>*)dw, (T)ih[0], (T)ih[1], (T)ih[2]);
  else
    hipLaunchKernelGGL((k_fine<2, SU, SF, SO, T, MODE>), grid1(thr), dim3(256), 0, s, g, (const SU*)u, (const SF*)f,
                       (SO*)out, (const cx<T>*)dg, (const cx<T>*)dw, (T)ih[0], (T)ih[1], (T)ih[2]);
}

template <class SU, class SF, class SO, class T>
static void fine_mode(int mode, int dim, const Geo& g, const void* u, const void* f, void* out, const void* dg,
                      const void* dw, const double ih[3], hipStream_t s) {
  switch (mode) {
    case 0: fine_dispatch<SU, SF, SO, T, 0>(dim, g, u, f, out, dg, dw, ih, s); break;
    case 1: fine_dispatch<SU, SF, SO, T, 1>(dim, g, u, f, out, dg, dw, ih, s); break;
    case 2: fine_dispatch<SU, SF, SO, T, 2>(dim, g, u, f, out, dg, dw, ih, s); break;
    default: fine_dispatch<SU, SF, SO, T, 3>(dim, g, u, f, out, dg, dw, ih, s); break;
  }
}

void launch_fine(int mode, Prec pu, Prec pf, Prec po, Prec pt, int dim, const Geo& g, const void* u, const void* f,
                 void* out, const void* dg, const void* dw, const double ih[3], hipStream_t s) {
  // Supported combinations: FP64 cycle / outer (c128 everywhere, double),
  // mixed cycle (c64 everywhere, float), outer apply of a c64 field into a
  // c128 result in double, and the FP32-basis outer products (c128 inputs or
  // c64 fields into c64 results, in double).
  if (pt == P64) {
    if (pu == P64 && pf == P64 && po == P64) return fine_mode<c128, c128, c128, double>(mode, dim, g, u, f, out, dg, dw, ih, s);
    if (pu == P32 && pf == P64 && po == P64) return fine_mode<c64, c128, c128, double>(mode, dim, g, u, f, out, dg, dw, ih, s);
    // FP32 outer basis: true residual from FP64 Q, X; W = H Z in FP64 arithmetic
    if (pu == P64 && pf == P64 && po == P32) return fine_mode<c128, c128, c64, double>(mode, dim, g, u, f, out, dg, dw, ih, s);
    if (pu == P32 && pf == P32 && po == P32) return fine_mode<c64, c64, c64, double>(mode, dim, g, u, f, out, dg, dw, ih, s);
  } else {
    if (pu == P32 && pf == P32 && po == P32) return fine_mode<c64, c64, c64, float>(mode, dim, g, u, f, out, dg, dw, ih, s);
    if (pu == P32 && pf == P64 && po == P32) return fine_mode<c64, c128, c64, float>(mode, dim, g, u, f, out, dg, dw, ih, s);
  }
  fatal_combo("launch_fine");
}

template <class S, class T, int MODE>
static void gal_dispatch(int dim, const Geo& g, const void* u, const void* f, void* out, const void* st,
                         const void* dw, hipStream_t s) {
  const int64_t thr = g.npts * (g.P / St<S>::R);
  if (dim == 3)
    hipLaunchKernelGGL((k_gal<3, S, T, MODE>), grid1(thr), dim3(256), 0, s, g, (const S*)u, (const S*)f, (S*)out,
                       (const cx<T>*)st, (const cx<T>*)dw);
  else
    hipLaunchKernelGGL((k_gal<2, S, T, MODE>), grid1(thr), dim3(256), 0, s, g, (const S*)u, (const S*)f, (S*)out,
                       (const cx<T>*)st, (const cx<T>*)dw);
}

template <class S, class T>
static void gal_mode(int mode, int dim, const Geo& g, const void* u, const void* f, void* out, const void* st,
                     const void* dw, hipStream_t s) {
  // the LDS-blocked family of tiles also takes the LDS form of the 27-point
  // stencil (bitwise the same results)
  if (dim == 3 && (g_tile.ry == 8 || g_tile.ry == 16) && mode != 3) {
    bool ran = false;
    switch (mode) {
      case 0: ran = gal_lds_launch<S, T, 0>(g, u, f, out, st, dw, s); break;
      case 1: ran = gal_lds_launch<S, T, 1>(g, u, f, out, st, dw, s); break;
      default: ran = gal_lds_launch<S, T, 2>(g, u, f, out, st, dw, s); break;
    }
    if (ran) return;
  }
  switch (mode) {
    case 0: gal_dispatch<S, T, 0>(dim, g, u, f, out, st, dw, s); break;
    case 1: gal_dispatch<S, T, 1>(dim, g, u, f, out, st, dw, s); break;
    case 2: gal_dispatch<S, T, 2>(dim, g, u, f, out, st, dw, s); break;
    default: gal_dispatch<S, T, 3>(dim, g, u, f, out, st, dw, s); break;
  }
}

void launch_gal(int mode, Prec ps, Prec pt, int dim, const Geo& g, const void* u, const void* f, void* out,
                const void* st, const void* dw, hipStream_t s) {
  if (ps == P64 && pt == P64) return gal_mode<c128, double>(mode, dim, g, u, f, out, st, dw, s);
  if (ps == P32 && pt == P32) return gal_mode<c64, float>(mode, dim, g, u, f, out, st, dw, s);
  if (ps == PBF && pt == P32) return gal_mode<cbf, float>(mode, dim, g, u, f, out, st, dw, s);
  fatal_combo("launch_gal");
}

template <class SI, class SO, class T>
static void restrict_t(int dim, const Geo& gf, const Geo& gc, const void* rf, void* rc, hipStream_t s) {
  constexpr int K = St<SI>::R > St<SO>::R ? St<SI>::R : St<SO>::R;
  const int64_t thr = gc.npts * (gc.P / K);
  if (dim == 3)
    hipLaunchKernelGGL((k_restrict<3, SI, SO, T>), grid1(thr), dim3(256), 0, s, gf, gc, (const SI*)rf, (SO*)rc);
  else
    hipLaunchKernelGGL((k_restrict<2, SI, SO, T>), grid1(thr), dim3(256), 0, s, gf, gc, (const SI*)rf, (SO*)rc);
}

void launch_restrict(Prec pi, Prec po, Prec pt, int dim, const Geo& gf, const Geo& gc, const void* rf, void* rc,
                     hipStream_t s) {
  if (pi == P64 && po == P64 && pt == P64) return restrict_t<c128, c128, double>(dim, gf, gc, rf, rc, s);
  if (pi == P32 && po == P32 && pt == P32) return restrict_t<c64, c64, float>(dim, gf, gc, rf, rc, s);
  if (pi == P32 && po == PBF && pt == P32) return restrict_t<c64, cbf, float>(dim, gf, gc, rf, rc, s);
  if (pi == PBF && po == PBF && pt == P32) return restrict_t<cbf, cbf, float>(dim, gf, gc, rf, rc, s);
  if (pi == PBF && po == P32 && pt == P32) return restrict_t<cbf, c64, float>(dim, gf, gc, rf, rc, s);
  fatal_combo("launch_restrict");
}

template <class SC, class SF, class T>
static void prolong_t(int dim, const Geo& gf, const Geo& gc, const void* ec, void* uf, hipStream_t s) {
  constexpr int K = St<SC>::R > St<SF>::R ? St<SC>::R : St<SF>::R;
  const int64_t thr = gf.npts * (gf.P / K);
  if (dim == 3)
    hipLaunchKernelGGL((k_prolong_add<3, SC, SF, T>), grid1(thr), dim3(256), 0, s, gf, gc, (const SC*)ec, (SF*)uf);
  else
    hipLaunchKernelGGL((k_prolong_add<2, SC, SF, T>), grid1(thr), dim3(256), 0, s, gf, gc, (const SC*)ec, (SF*)uf);
}

void launch_prolong_add(Prec pc, Prec pf, Prec pt, int dim, const Geo& gf, const Geo& gc, const void* ec, void* uf,
                        hipStream_t s) {
  if (pc == P64 && pf == P64 && pt == P64) return prolong_t<c128, c128, double>(dim, gf, gc, ec, uf, s);
  if (pc == P32 && pf == P32 && pt == P32) return prolong_t<c64, c64, float>(dim, gf, gc, ec, uf, s);
  if (pc == PBF && pf == P32 && pt == P32) return prolong_t<cbf, c64, float>(dim, gf, gc, ec, uf, s);
  if (pc == PBF && pf == PBF && pt == P32) return prolong_t<cbf, cbf, float>(dim, gf, gc, ec, uf, s);
  if (pc == P32 && pf == PBF && pt == P32) return prolong_t<c64, cbf, float>(dim, gf, gc, ec, uf, s);
  fatal_combo("launch_prolong_add");
}

void launch_convert(Prec pi, Prec po, int64_t nvals, const void* a, void* b, hipStream_t s) {
  if (pi == P64 && po == P32)
    { hipLaunchKernelGGL((k_convert<c128, c64, double>), grid1(nvals / 2), dim3(256), 0, s, nvals, (const c128*)a, (c64*)b); return; }
  if (pi == P32 && po == P64)
    { hipLaunchKernelGGL((k_convert<c64, c128, double>), grid1(nvals / 2), dim3(256), 0, s, nvals, (const c64*)a, (c128*)b); return; }
  if (pi == P32 && po == PBF)
    { hipLaunchKernelGGL((k_convert<c64, cbf, float>), grid1(nvals / 4), dim3(256), 0, s, nvals, (const c64*)a, (cbf*)b); return; }
  if (pi == PBF && po == P32)
    { hipLaunchKernelGGL((k_convert<cbf, c64, float>), grid1(nvals / 4), dim3(256), 0, s, nvals, (const cbf*)a, (c64*)b); return; }
  if (pi == P64 && po == PBF)
    { hipLaunchKernelGGL((k_convert<c128, cbf, double>), grid1(nvals / 4), dim3(256), 0, s, nvals, (const c128*)a, (cbf*)b); return; }
  if (pi == PBF && po == P64)
    { hipLaunchKernelGGL((k_convert<cbf, c128, double>), grid1(nvals / 4), dim3(256), 0, s, nvals, (const cbf*)a, (c128*)b); return; }
  fatal_combo("launch_convert");
}

// z1 <- y1 z1 + y2 z2 per column c (y_j of column c at Y[j * P + c]), the
// K-cycle's combination of its two preconditioned vectors; FP64 arithmetic,
// rounded once to the field's storage.
template <class S>
__global__ void k_kc_combine(int64_t n, int P, const c128* __restrict__ Y, S* __restrict__ z1,
                             const S* __restrict__ z2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = (int)(i % P);
  const c128 a = get1(z1 + i), b = get1(z2 + i);
  const c128 y1 = Y[c], y2 = Y[(int64_t)P + c];
  put1(z1 + i, c128{y1.re * a.re - y1.im * a.im + (y2.re * b.re - y2.im * b.im),
                    y1.re * a.im + y1.im * a.re + (y2.re * b.im + y2.im * b.re)});
}

void launch_kc_combine(Prec pf, int64_t N, int P, const c128* Y, void* z1, const void* z2, hipStream_t s) {
  const int64_t n = N * P;
  if (pf == P64)
    hipLaunchKernelGGL((k_kc_combine<c128>), grid1(n), dim3(256), 0, s, n, P, Y, (c128*)z1, (const c128*)z2);
  else if (pf == P32)
    hipLaunchKernelGGL((k_kc_combine<c64>), grid1(n), dim3(256), 0, s, n, P, Y, (c64*)z1, (const c64*)z2);
  else
    hipLaunchKernelGGL((k_kc_combine<cbf>), grid1(n), dim3(256), 0, s, n, P, Y, (cbf*)z1, (const cbf*)z2);
}

void launch_to_internal(Prec po, int64_t N, int nrhs, int P, const void* src, void* dst, hipStream_t s) {
  dim3 gr((unsigned)((N + 31) / 32), (unsigned)((P + 31) / 32));
  if (po == P64) { hipLaunchKernelGGL((k_to_internal<c128>), gr, dim3(256), 0, s, N, nrhs, P, (const c128*)src, (c128*)dst); return; }
  if (po == P32) { hipLaunchKernelGGL((k_to_internal<c64>), gr, dim3(256), 0, s, N, nrhs, P, (const c128*)src, (c64*)dst); return; }
  { hipLaunchKernelGGL((k_to_internal<cbf>), gr, dim3(256), 0, s, N, nrhs, P, (const c128*)src, (cbf*)dst); return; }
}

void launch_to_abi(Prec pi, int64_t N, int nrhs, int P, const void* src, void* dst, hipStream_t s) {
  dim3 gr((unsigned)((N + 31) / 32), (unsigned)((P + 31) / 32));
  if (pi == P64) { hipLaunchKernelGGL((k_to_abi<c128>), gr, dim3(256), 0, s, N, nrhs, P, (const c128*)src, (c128*)dst); return; }
  if (pi == P32) { hipLaunchKernelGGL((k_to_abi<c64>), gr, dim3(256), 0, s, N, nrhs, P, (const c64*)src, (c128*)dst); return; }
  { hipLaunchKernelGGL((k_to_abi<cbf>), gr, dim3(256), 0, s, N, nrhs, P, (const cbf*)src, (c128*)dst); return; }
}

// ---------------------------------------------------------------------------
// Persistent cycle. One cooperative launch runs the recorded phases of a
// cycle in order: the items of a phase are dealt out grid-stride (GEMM tiles
// one per workgroup in turn) and every workgroup waits at a grid barrier
// before the next phase reads what the previous one wrote. Each phase runs
// the per-item code of the stand-alone kernel, so the arithmetic is that of
// the eager generic kernels.
// ---------------------------------------------------------------------------
template <int DIM, class S, class T>
__device__ void ph_fine(const Phase& q, int64_t t0, int64_t gs) {
  const int64_t n = q.g.npts * (q.g.P / St<S>::R);
  const T hx = (T)q.ih[0], hy = (T)q.ih[1], hz = (T)q.ih[2];
  const S* u = static_cast<const S*>(q.u);
  const S* f = static_cast<const S*>(q.f);
  S* o = static_cast<S*>(q.out);
  const cx<T>* dg = static_cast<const cx<T>*>(q.c0);
  const cx<T>* dw = static_cast<const cx<T>*>(q.c1);
  switch (q.mode) {
    case 0:
      for (int64_t t = t0; t < n; t += gs) fine_item<DIM, S, S, S, T, 0>(q.g, t, u, f, o, dg, dw, hx, hy, hz);
      break;
    case 1:
      for (int64_t t = t0; t < n; t += gs) fine_item<DIM, S, S, S, T, 1>(q.g, t, u, f, o, dg, dw, hx, hy, hz);
      break;
    case 2:
      for (int64_t t = t0; t < n; t += gs) fine_item<DIM, S, S, S, T, 2>(q.g, t, u, f, o, dg, dw, hx, hy, hz);
      break;
    default:
      for (int64_t t = t0; t < n; t += gs) fine_item<DIM, S, S, S, T, 3>(q.g, t, u, f, o, dg, dw, hx, hy, hz);
      break;
  }
}

template <int DIM, class S, class T>
__device__ void ph_gal(const Phase& q, int64_t t0, int64_t gs) {
  const int64_t n = q.g.npts * (q.g.P / St<S>::R);
  const S* u = static_cast<const S*>(q.u);
  const S* f = static_cast<const S*>(q.f);
  S* o = static_cast<S*>(q.out);
  const cx<T>* st = static_cast<const cx<T>*>(q.c0);
  const cx<T>* dw = static_cast<const cx<T>*>(q.c1);
  switch (q.mode) {
    case 0: for (int64_t t = t0; t < n; t += gs) gal_item<DIM, S, T, 0>(q.g, t, u, f, o, st, dw); break;
    case 1: for (int64_t t = t0; t < n; t += gs) gal_item<DIM, S, T, 1>(q.g, t, u, f, o, st, dw); break;
    case 2: for (int64_t t = t0; t < n; t += gs) gal_item<DIM, S, T, 2>(q.g, t, u, f, o, st, dw); break;
    default: for (int64_t t = t0; t < n; t += gs) gal_item<DIM, S, T, 3>(q.g, t, u, f, o, st, dw); break;
  }
}

template <int DIM, class SI, class SO, class T>
__device__ void ph_restrict(const Phase& q, int64_t t0, int64_t gs) {
  constexpr int K = St<SI>::R > St<SO>::R ? St<SI>::R : St<SO>::R;
  const int64_t n = q.gc.npts * (q.gc.P / K);
  for (int64_t t = t0; t < n; t += gs)
    restrict_item<DIM, SI, SO, T>(q.g, q.gc, t, static_cast<const SI*>(q.u), static_cast<SO*>(q.out));
}

template <int DIM, class SC, class SF, class T>
__device__ void ph_prolong(const Phase& q, int64_t t0, int64_t gs) {
  constexpr int K = St<SC>::R > St<SF>::R ? St<SC>::R : St<SF>::R;
  const int64_t n = q.g.npts * (q.g.P / K);
  for (int64_t t = t0; t < n; t += gs)
    prolong_item<DIM, SC, SF, T>(q.g, q.gc, t, static_cast<const SC*>(q.u), static_cast<SF*>(q.out));
}

// out = A B for the coarsest level: A the n x n inverse, B and out [n][P]
template <class S, class T>
__device__ void ph_gemm(const Phase& q, cx<T> (&As)[GEMM_BK][GEMM_BM + 1], cx<T> (&Bs)[GEMM_BK][GEMM_BN + 1]) {
  const int64_t M = q.n, N = q.g.P;
  const int64_t gx = (N + GEMM_BN - 1) / GEMM_BN, ntiles = gx * ((M + GEMM_BM - 1) / GEMM_BM);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
    gemm_tile<S, T>((unsigned)(tile % gx), (unsigned)(tile / gx), M, N, M, cx<T>{(T)1, (T)0},
                    static_cast<const S*>(q.c0), M, static_cast<const S*>(q.u), N, cx<T>{(T)0, (T)0},
                    static_cast<S*>(q.out), N, As, Bs);
}

template <int DIM, bool MIX>
__global__ __launch_bounds__(256) void k_cycle_persist(const Phase* __restrict__ ph, int nph) {
  using T = typename std::conditional<MIX, float, double>::type;
  __shared__ cx<T> As[GEMM_BK][GEMM_BM + 1];
  __shared__ cx<T> Bs[GEMM_BK][GEMM_BN + 1];
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  const int64_t gs = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int p = 0; p < nph; ++p) {
    const Phase q = ph[p];
    if (q.op == PH_FINE) {
      if constexpr (MIX) ph_fine<DIM, c64, float>(q, t0, gs);
      else ph_fine<DIM, c128, double>(q, t0, gs);
    } else if (q.op == PH_GAL) {
      if constexpr (MIX) {
        if (q.pa == PBF) ph_gal<DIM, cbf, float>(q, t0, gs);
        else ph_gal<DIM, c64, float>(q, t0, gs);
      } else {
        ph_gal<DIM, c128, double>(q, t0, gs);
      }
    } else if (q.op == PH_RESTRICT) {
      if constexpr (MIX) {
        if (q.pa == P32 && q.pb == PBF) ph_restrict<DIM, c64, cbf, float>(q, t0, gs);
        else if (q.pa == PBF && q.pb == PBF) ph_restrict<DIM, cbf, cbf, float>(q, t0, gs);
        else if (q.pa == PBF && q.pb == P32) ph_restrict<DIM, cbf, c64, float>(q, t0, gs);
        else ph_restrict<DIM, c64, c64, float>(q, t0, gs);
      } else {
        ph_restrict<DIM, c128, c128, double>(q, t0, gs);
      }
    } else if (q.op == PH_PROLONG) {
      if constexpr (MIX) {
        if (q.pa == PBF && q.pb == P32) ph_prolong<DIM, cbf, c64, float>(q, t0, gs);
        else if (q.pa == PBF && q.pb == PBF) ph_prolong<DIM, cbf, cbf, float>(q, t0, gs);
        else if (q.pa == P32 && q.pb == PBF) ph_prolong<DIM, c64, cbf, float>(q, t0, gs);
        else ph_prolong<DIM, c64, c64, float>(q, t0, gs);
      } else {
        ph_prolong<DIM, c128, c128, double>(q, t0, gs);
      }
    } else if (q.op == PH_ZERO) {
      uint4* o = static_cast<uint4*>(q.out);
      for (int64_t t = t0; t < q.n; t += gs) o[t] = uint4{0u, 0u, 0u, 0u};
    } else if (q.op == PH_GEMM) {
      if constexpr (MIX) ph_gemm<c64, float>(q, As, Bs);
      else ph_gemm<c128, double>(q, As, Bs);
    }
    grid.sync();
  }
}

template <int DIM, bool MIX> static int persist_grid_t() {
  static const int g = [] {
    int dev = 0, cus = 0, nb = 0, coop = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_cycle_persist<DIM, MIX>, 256, 0) != hipSuccess)
      return 0;
    return nb * cus;
  }();
  return g;
}

int persist_grid(int dim, bool mixed) {
  if (dim == 3) return mixed ? persist_grid_t<3, true>() : persist_grid_t<3, false>();
  return mixed ? persist_grid_t<2, true>() : persist_grid_t<2, false>();
}

template <int DIM, bool MIX>
static hipError_t persist_launch(const Phase* ph, int nph, int grid, hipStream_t s) {
  void* args[] = {(void*)&ph, (void*)&nph};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_cycle_persist<DIM, MIX>), dim3((unsigned)grid),
                                    dim3(256), args, 0, s);
}

hipError_t launch_cycle_persist(int dim, bool mixed, const Phase* ph, int nph, int grid, hipStream_t s) {
  if (grid < 1 || grid > persist_grid(dim, mixed)) return hipErrorInvalidValue;
  if (dim == 3) return mixed ? persist_launch<3, true>(ph, nph, grid, s) : persist_launch<3, false>(ph, nph, grid, s);
  return mixed ? persist_launch<2, true>(ph, nph, grid, s) : persist_launch<2, false>(ph, nph, grid, s);
}

}  // namespace helm
