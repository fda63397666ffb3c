// tile_gemm.hpp -- one 64 x 64 output tile of a complex GEMM, shared by the
// stand-alone GEMM kernel and the persistent cycle (same arithmetic order).
#pragma once
#include "common.hpp"

namespace helm {

// C = alpha A B + beta C, row-major. The 256-lane workgroup computes the
// 64x64 tile (tile row by, tile column bx); each lane a 4x4 sub-tile (rows
// ty+16r, cols tx+16c), K staged through LDS in steps of 8. Every lane of the
// workgroup must call it (it synchronises the workgroup).
constexpr int GEMM_BM = 64, GEMM_BN = 64, GEMM_BK = 8;
template <class S, class T>
__device__ __forceinline__ void gemm_tile(unsigned bx, unsigned by, int64_t M, int64_t N, int64_t K, cx<T> alpha,
                                          const S* __restrict__ A, int64_t lda, const S* __restrict__ B,
                                          int64_t ldb, cx<T> beta, S* __restrict__ C, int64_t ldc,
                                          cx<T> (&As)[GEMM_BK][GEMM_BM + 1], cx<T> (&Bs)[GEMM_BK][GEMM_BN + 1]) {
  constexpr int BM = GEMM_BM, BN = GEMM_BN, BK = GEMM_BK;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t m0 = (int64_t)by * BM, n0 = (int64_t)bx * BN;
  cx<T> acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = {(T)0, (T)0};
  for (int64_t k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int idx = threadIdx.x + 256 * e;  // 512 = BM*BK
      const int am = idx / BK, ak = idx % BK;
      const int64_t gm = m0 + am, gk = k0 + ak;
      cx<T> v = {(T)0, (T)0};
      if (gm < M && gk < K) {
        const S a = A[gm * lda + gk];
        v = {(T)a.re, (T)a.im};
      }
      As[ak][am] = v;
      const int bk = idx / BN, bn = idx % BN;
      const int64_t hk = k0 + bk, hn = n0 + bn;
      cx<T> w = {(T)0, (T)0};
      if (hk < K && hn < N) {
        const S b = B[hk * ldb + hn];
        w = {(T)b.re, (T)b.im};
      }
      Bs[bk][bn] = w;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      cx<T> a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = As[kk][ty + 16 * r];
#pragma unroll
      for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tx + 16 * c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) cfma(acc[r][c], a[r], b[c]);
    }
    __syncthreads();
  }
  const bool bz = beta.re == (T)0 && beta.im == (T)0;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int64_t gm = m0 + ty + 16 * r, gn = n0 + tx + 16 * c;
      if (gm < M && gn < N) {
        cx<T> v = alpha * acc[r][c];
        if (!bz) {
          const S o = C[gm * ldc + gn];
          v = v + beta * cx<T>{(T)o.re, (T)o.im};
        }
        C[gm * ldc + gn] = S{v.re, v.im};
      }
    }
}

}  // namespace helm
