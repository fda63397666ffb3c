// k_bicg.hip -- the small per-group steps of block BiCGSTAB (El Guennouni,
// Jbilou and Sadok's block version, the paper's W-BiCG solver of section
// 5.3): the pb x pb solves for alpha and beta, the scalar omega, and the
// coefficient lists that let the block-update kernel of k_krylov.hip form
// S, X, R and P in one pass each. The tall-skinny products (Gram blocks and
// updates over N points) are k_krylov.hip's.
//
// Matrices of a group g (columns g*pb .. g*pb+pb-1 of the block) are kept
// in the Gram layout: M[a][b] at index (g*pb + b)*pb + a. A Gram product
// of the shadow block Rt with Y gives (Rt_g^H Y_g)[a][b] in that layout,
// and a coefficient C in that layout is what launch_block_update applies:
// Y[n][g*pb+b] (+/-)= sum_a X[n][g*pb+a] C[a][b].
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace helm {

__device__ inline cx<double> tcd(const c128& v) { return cx<double>{v.re, v.im}; }
__device__ inline c128 fcd(const cx<double>& v) { return c128{v.re, v.im}; }

// X_g = sgn * A_g^-1 B_g per group (one workgroup each) by Gaussian
// elimination with partial pivoting; an inactive group, or a pivot below
// 1e-13 of the largest entry of A_g (flag[g] = 1), gives X_g = 0. The group
// size is at most BICG_MAXPB (the block-size limit of the solver); the four
// working matrices take 128 KB of static LDS at 64 columns (gfx950 gives a
// workgroup up to 160 KB).
constexpr int BICG_MAXPB = 64;
__global__ __launch_bounds__(64) void k_bicg_solve(int pb, double sgn, const c128* __restrict__ A,
                                                   const c128* __restrict__ B, c128* __restrict__ X,
                                                   const int* __restrict__ act, int* __restrict__ flag) {
  __shared__ double Mr[BICG_MAXPB * BICG_MAXPB], Mi[BICG_MAXPB * BICG_MAXPB];
  __shared__ double Rr[BICG_MAXPB * BICG_MAXPB], Ri[BICG_MAXPB * BICG_MAXPB];
  __shared__ int bad;
  __shared__ double amax;
  const int g = blockIdx.x, tid = threadIdx.x;
  const int64_t o = (int64_t)g * pb * pb;
  for (int e = tid; e < pb * pb; e += blockDim.x) {
    const int a = e / pb, b = e % pb;
    const c128 av = A[o + (int64_t)b * pb + a], bv = B[o + (int64_t)b * pb + a];
    Mr[e] = av.re;
    Mi[e] = av.im;
    Rr[e] = bv.re;
    Ri[e] = bv.im;
  }
  if (tid == 0) {
    bad = act[g] ? 0 : 2;
    amax = 0.0;
  }
  __syncthreads();
  if (tid == 0 && !bad)
    for (int e = 0; e < pb * pb; ++e) amax = fmax(amax, sqrt(Mr[e] * Mr[e] + Mi[e] * Mi[e]));
  __syncthreads();
  for (int k = 0; k < pb && !bad; ++k) {
    if (tid == 0) {
      int piv = k;
      double best = -1.0;
      for (int a = k; a < pb; ++a) {
        const double v = Mr[a * pb + k] * Mr[a * pb + k] + Mi[a * pb + k] * Mi[a * pb + k];
        if (v > best) {
          best = v;
          piv = a;
        }
      }
      if (!(sqrt(best) > 1e-13 * amax)) bad = 1;
      if (piv != k && !bad)
        for (int b = 0; b < pb; ++b) {
          double t = Mr[k * pb + b];
          Mr[k * pb + b] = Mr[piv * pb + b];
          Mr[piv * pb + b] = t;
          t = Mi[k * pb + b];
          Mi[k * pb + b] = Mi[piv * pb + b];
          Mi[piv * pb + b] = t;
          t = Rr[k * pb + b];
          Rr[k * pb + b] = Rr[piv * pb + b];
          Rr[piv * pb + b] = t;
          t = Ri[k * pb + b];
          Ri[k * pb + b] = Ri[piv * pb + b];
          Ri[piv * pb + b] = t;
        }
    }
    __syncthreads();
    if (bad) break;
    // eliminate below the pivot (rows a > k), one row per lane
    const double pr = Mr[k * pb + k], pi = Mi[k * pb + k];
    const double pd = pr * pr + pi * pi;
    for (int a = k + 1 + tid; a < pb; a += blockDim.x) {
      const double xr = Mr[a * pb + k], xi = Mi[a * pb + k];
      const double lr = (xr * pr + xi * pi) / pd, li = (xi * pr - xr * pi) / pd;  // l = x / pivot
      for (int b = k; b < pb; ++b) {
        const double mr = Mr[k * pb + b], mi = Mi[k * pb + b];
        Mr[a * pb + b] -= lr * mr - li * mi;
        Mi[a * pb + b] -= lr * mi + li * mr;
      }
      for (int b = 0; b < pb; ++b) {
        const double rr = Rr[k * pb + b], ri = Ri[k * pb + b];
        Rr[a * pb + b] -= lr * rr - li * ri;
        Ri[a * pb + b] -= lr * ri + li * rr;
      }
    }
    __syncthreads();
  }
  if (bad) {
    for (int e = tid; e < pb * pb; e += blockDim.x) X[o + e] = c128{0.0, 0.0};
    if (tid == 0) flag[g] = bad == 1 ? 1 : 0;
    return;
  }
  // back substitution, one right-hand-side column per lane
  for (int b = tid; b < pb; b += blockDim.x) {
    for (int a = pb - 1; a >= 0; --a) {
      double sr = Rr[a * pb + b], si = Ri[a * pb + b];
      for (int l = a + 1; l < pb; ++l) {
        const double mr = Mr[a * pb + l], mi = Mi[a * pb + l], xr = Rr[l * pb + b], xi = Ri[l * pb + b];
        sr -= mr * xr - mi * xi;
        si -= mr * xi + mi * xr;
      }
      const double dr = Mr[a * pb + a], di = Mi[a * pb + a], dd = dr * dr + di * di;
      Rr[a * pb + b] = (sr * dr + si * di) / dd;
      Ri[a * pb + b] = (si * dr - sr * di) / dd;
    }
  }
  __syncthreads();
  for (int e = tid; e < pb * pb; e += blockDim.x) {
    const int a = e / pb, b = e % pb;
    X[o + (int64_t)b * pb + a] = c128{sgn * Rr[e], sgn * Ri[e]};
  }
  if (tid == 0) flag[g] = 0;
}

void launch_bicg_solve(int ng, int pb, double sgn, const c128* A, const c128* B, c128* X, const int* act, int* flag,
                       hipStream_t s) {
  if (pb < 1 || pb > BICG_MAXPB) fatal_combo("launch_bicg_solve");
  hipLaunchKernelGGL(k_bicg_solve, dim3(ng), dim3(64), 0, s, pb, sgn, A, B, X, act, flag);
}

// omega_g = sum_b (T^H S)[b][b] / sum_b ||T_b||^2 over the group's columns
// (Gts in the Gram layout of [T] against S, tn2 per column); 0 for an
// inactive group or a zero T.
__global__ void k_bicg_omega(int ng, int pb, const c128* __restrict__ Gts, const double* __restrict__ tn2,
                             const int* __restrict__ act, c128* __restrict__ om) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ng) return;
  cx<double> num = {0.0, 0.0};
  double den = 0.0;
  for (int b = 0; b < pb; ++b) {
    const int c = g * pb + b;
    num = num + tcd(Gts[(int64_t)c * pb + b]);
    den += tn2[c];
  }
  om[g] = act[g] && den > 0.0 ? c128{num.re / den, num.im / den} : c128{0.0, 0.0};
}

void launch_bicg_omega(int ng, int pb, const c128* Gts, const double* tn2, const int* act, c128* om, hipStream_t s) {
  hipLaunchKernelGGL(k_bicg_omega, dim3((ng + 63) / 64), dim3(64), 0, s, ng, pb, Gts, tn2, act, om);
}

// Coefficient lists for launch_block_update, k matrices of P*pb entries
// each in the Gram layout (I: identity of the group, om: omega_g):
//   kind 0 (S = R - V alpha, X list [V, R], overwrite):   [-alpha, I]
//   kind 1 (X += Phat alpha + omega Shat, [Phat, Shat]):  [alpha, om I]
//   kind 2 (R = S - omega T, [S, T], overwrite):          [I, -om I]
//   kind 3 (P = R + (P - omega V) beta, [R, P, V]):       [I, beta, -om beta]
__global__ void k_bicg_coefs(int kind, int P, int pb, const c128* __restrict__ M, const c128* __restrict__ om,
                             c128* __restrict__ C) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)P * pb;
  if (e >= n) return;
  const int c = (int)(e / pb), a = (int)(e % pb);
  const int g = c / pb, b = c % pb;
  const cx<double> m = M ? tcd(M[e]) : cx<double>{0.0, 0.0};
  const cx<double> w = tcd(om[g]);
  const cx<double> id = {a == b ? 1.0 : 0.0, 0.0};
  switch (kind) {
    case 0:
      C[e] = fcd(cx<double>{-m.re, -m.im});
      C[n + e] = fcd(id);
      break;
    case 1:
      C[e] = fcd(m);
      C[n + e] = fcd(w * id);
      break;
    case 2:
      C[e] = fcd(id);
      C[n + e] = fcd(cx<double>{-w.re, -w.im} * id);
      break;
    default:
      C[e] = fcd(id);
      C[n + e] = fcd(m);
      C[2 * n + e] = fcd(cx<double>{-w.re, -w.im} * m);
      break;
  }
}

void launch_bicg_coefs(int kind, int P, int pb, const c128* M, const c128* om, c128* C, hipStream_t s) {
  const int64_t n = (int64_t)P * pb;
  hipLaunchKernelGGL(k_bicg_coefs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, kind, P, pb, M, om, C);
}

}  // namespace helm
