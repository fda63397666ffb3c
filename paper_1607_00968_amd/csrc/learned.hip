// learned.hip -- learned coarsest-grid correction: a small convolutional
// network maps the coarsest-grid residual to an approximation of the
// coarsest-grid error, replacing the coarsest solve inside the cycle.
//
// The paper names a stationary inexact solver of the coarsest grid as the
// direction of its future work (end of section 5.3 and the conclusions);
// this network is one. Architecture: a 3-level U-Net on a D^3 volume
// (D = coarsest unknowns per axis rounded up to a multiple of 4), channels
// last, BF16 activations and weights, FP32 accumulation and master weights:
//   enc: conv3(4->16) conv3(16->16)=s1 | pool | conv3(16->32) conv3(32->32)=s2
//        | pool | conv3(32->64) conv3(64->64)
//   dec: up, concat s2 -> conv3(96->32) conv3(32->32) | up, concat s1 ->
//        conv3(48->16) conv3(16->16) | 1x1 head 16->2 (linear)
// Input channels: Re, Im of r / rms(r), and Re, Im of H^2 diag(M_c) (the
// coarse operator's diagonal: carries the slowness and the absorbing layer).
// Output: e = H^2 rms(r) (out_0 + i out_1).
//
// 3x3x3 convolutions run as implicit GEMMs on the matrix cores
// (v_mfma_f32_16x16x16_bf16): M = voxels, N = output channels, K = 27 x
// input channels; the backward-data pass is the same kernel with mirrored
// taps and transposed weights. Weight gradients accumulate in FP32 per chunk
// of voxels and are summed in a fixed order (deterministic).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "kernels.hpp"
#include "learned.hpp"

namespace helm {
namespace learned {

typedef uint16_t bf16;
typedef short short4_ __attribute__((ext_vector_type(4)));
typedef float float4_ __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int NLAYER = 10;
constexpr int L_CIN[NLAYER] = {4, 16, 16, 32, 32, 64, 96, 32, 48, 16};
constexpr int L_COUT[NLAYER] = {16, 16, 32, 32, 64, 64, 32, 32, 16, 16};

static int64_t layer_off(int l) {
  int64_t o = 0;
  for (int k = 0; k < l; ++k) o += 27LL * L_CIN[k] * L_COUT[k] + L_COUT[k];
  return o;
}
static int64_t nparams_total() { return layer_off(NLAYER) + 16 * 2 + 2; }

__device__ inline float b2f(bf16 b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }

// ---------------------------------------------------------------------------
// 3x3x3 convolution as an implicit GEMM on MFMA 16x16x16 (bf16 in, f32 acc).
// Lane l of a wave supplies A[m = l%16][k = 4(l/16)..+3] (four consecutive
// input channels of one tap), B[k][n = l%16] and receives
// D[m = 4(l/16)+j][n = l%16]. A wave owns 32 voxels (two M tiles) and all
// NT*16 output channels; a workgroup of four waves owns 128 voxels.
// ---------------------------------------------------------------------------
struct ConvArgs {
  int B, D, Cin, N;
  const bf16* in;
  int ldi, offi;
  const bf16* W;  // [27][N][Cin]
  const float* bias;
  bf16* out;
  int ldo, offo;
  int flip, relu;
  const bf16* mask;  // out *= (mask[v][offm + n] > 0) when set
  int ldm, offm;
  // A second input (the 16- and 32-channel kernels only): when in2 is set,
  // input channels [C1, Cin) are channels [0, Cin - C1) of in2 (row stride
  // ldi2), and channels [0, C1) come from in; with up1, in holds a grid of
  // half the edge and voxel (x, y, z) reads its voxel (x/2, y/2, z/2), the
  // nearest upsampling. A decoder layer thus reads its skip input and the
  // upsampled coarser activations where they are, with no concatenated copy.
  const bf16* in2;
  int ldi2, C1, up1;
};

template <int NT>
__global__ __launch_bounds__(256) void k_conv3(ConvArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t V = (int64_t)a.D * a.D * a.D;
  const int64_t total = (int64_t)a.B * V;
  const int64_t vbase = (int64_t)blockIdx.x * 128 + wave * 32;
  const int ml = lane & 15, kg = lane >> 4;
  // coordinates of the two voxels this lane feeds into A
  int64_t gv[2];
  int vx[2], vy[2], vz[2];
  bool vin[2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    gv[mt] = vbase + mt * 16 + ml;
    vin[mt] = gv[mt] < total;
    const int64_t v = vin[mt] ? gv[mt] % V : 0;
    vx[mt] = (int)(v % a.D);
    vy[mt] = (int)((v / a.D) % a.D);
    vz[mt] = (int)(v / ((int64_t)a.D * a.D));
  }
  float4_ acc[2][NT];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = float4_{0.f, 0.f, 0.f, 0.f};
  const int Ktot = 27 * a.Cin;
  const int sgn = a.flip ? -1 : 1;
  for (int k0 = 0; k0 < Ktot; k0 += 16) {
    const int k = k0 + 4 * kg;
    const bool kin = k < Ktot;
    const int tap = kin ? k / a.Cin : 0;
    const int ci = kin ? k - tap * a.Cin : 0;
    const int dx = sgn * (tap % 3 - 1), dy = sgn * ((tap / 3) % 3 - 1), dz = sgn * (tap / 9 - 1);
    short4_ A[2], Bv[NT];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const int x = vx[mt] + dx, y = vy[mt] + dy, z = vz[mt] + dz;
      const bool ok = kin && vin[mt] && x >= 0 && x < a.D && y >= 0 && y < a.D && z >= 0 && z < a.D;
      if (ok) {
        const int64_t nb = gv[mt] + dx + (int64_t)a.D * (dy + (int64_t)a.D * dz);
        A[mt] = *reinterpret_cast<const short4_*>(a.in + nb * a.ldi + a.offi + ci);
      } else {
        A[mt] = short4_{0, 0, 0, 0};
      }
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int n = nt * 16 + ml;
      Bv[nt] = kin ? *reinterpret_cast<const short4_*>(a.W + ((int64_t)tap * a.N + n) * a.Cin + ci)
                   : short4_{0, 0, 0, 0};
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[mt], Bv[nt], acc[mt][nt], 0, 0, 0);
  }
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t v = vbase + mt * 16 + 4 * kg + j;
      if (v >= total) continue;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int n = nt * 16 + ml;
        float r = acc[mt][nt][j] + (a.bias ? a.bias[n] : 0.f);
        if (a.relu && !(r > 0.f)) r = 0.f;
        if (a.mask && !(b2f(a.mask[v * a.ldm + a.offm + n]) > 0.f)) r = 0.f;
        a.out[v * a.ldo + a.offo + n] = f2bf(r);
      }
    }
}

// LDS-tiled form for Cin % 16 == 0: a workgroup owns an 8x8x4 block of
// output voxels of one sample. Per chunk of 16 input channels it stages the
// 10x10x6 input halo (16 B per voxel and half chunk) and, one z-plane of taps
// at a time, the weights of 9 taps in LDS; the 27 tap products then read
// only LDS. Wave w owns output plane z = w of the block (four 16-voxel M
// tiles) and all NT*16 output channels. Tiles are numbered so that
// consecutive tiles of a sample land on one XCD (shared halo in its L2).
constexpr int CT_X = 8, CT_Y = 8, CT_Z = 4;
constexpr int CH_X = CT_X + 2, CH_Y = CT_Y + 2, CH_Z = CT_Z + 2, CH_V = CH_X * CH_Y * CH_Z;
constexpr int CCH = 16;
// LDS layout of the halo and the weights, chosen for the A and B fragment
// reads (8 B per lane; a 32-lane pass spans 16 rows of 32 B for two lane
// groups kg): an A fragment's 16 voxels are two x-rows of 8, 10 voxels apart,
// and at 32 B per voxel both rows fell on the same 32 banks. Each halo row of
// CH_X voxels is therefore followed by 16 B of padding, which moves the
// second row to the other 32 banks. A B fragment's 16 weight rows (32 B
// each) wrapped the same way; rows 8..15 of every 16 keep their two 16-B
// halves swapped. The values and the MFMA order are unchanged.
constexpr int CH_PAD_U4 = CH_V * 2 + CH_Y * CH_Z;  // halo size in 16-B units
__device__ inline int halo_u4(int hv) { return hv * 2 + hv / CH_X; }
// bf16 offset of voxel v (row r = v / CH_X) of the padded halo
__device__ inline int halo_el(int v, int r) { return v * CCH + r * 8; }
// bf16 offset of 8-B chunk kg of weight row `row` (rows 8..15 of each 16 swapped)
__device__ inline int wrow_el(int row, int kg) { return row * CCH + 4 * (kg ^ (((row >> 3) & 1) << 1)); }
__device__ inline int wrow_u4(int row, int half) { return row * 2 + (half ^ ((row >> 3) & 1)); }

template <int NT>
__global__ __launch_bounds__(256) void k_conv3_lds(ConvArgs a, int ntx, int nty, int ntz, int64_t ntiles,
                                                   int64_t per) {
  extern __shared__ uint4 lds_u4[];
  bf16* xs = reinterpret_cast<bf16*>(lds_u4);  // [CH_V][CCH], rows padded
  bf16* ws = xs + CH_PAD_U4 * 8;               // [9][N][CCH]
  constexpr int N = NT * 16;
  const int64_t t = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (t >= ntiles) return;  // whole workgroup leaves together
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ml = lane & 15, kg = lane >> 4;
  const int D = a.D;
  int64_t r = t;
  const int tx = (int)(r % ntx);
  r /= ntx;
  const int ty = (int)(r % nty);
  r /= nty;
  const int tz = (int)(r % ntz);
  const int64_t b = r / ntz;
  const int x0 = tx * CT_X, y0 = ty * CT_Y, z0 = tz * CT_Z;
  const int64_t sbase = b * (int64_t)D * D * D;
  int hb[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const int q = (wave * 4 + mt) * 16 + ml;
    hb[mt] = (q % CT_X + 1) + CH_X * ((q / CT_X) % CT_Y + 1 + CH_Y * (q / (CT_X * CT_Y) + 1));
  }
  float4_ acc[4][NT];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = float4_{0.f, 0.f, 0.f, 0.f};
  const int sgn = a.flip ? -1 : 1;
  for (int c0 = 0; c0 < a.Cin; c0 += CCH) {
    for (int pz = 0; pz < 3; ++pz) {
      __syncthreads();
      if (pz == 0) {
        for (int e = threadIdx.x; e < CH_V * 2; e += 256) {
          const int hv = e >> 1, half = e & 1;
          const int gx = x0 + hv % CH_X - 1, gy = y0 + (hv / CH_X) % CH_Y - 1, gz = z0 + hv / (CH_X * CH_Y) - 1;
          uint4 val{0u, 0u, 0u, 0u};
          if (gx >= 0 && gx < D && gy >= 0 && gy < D && gz >= 0 && gz < D)
            val = *reinterpret_cast<const uint4*>(a.in + (sbase + gx + (int64_t)D * (gy + (int64_t)D * gz)) * a.ldi +
                                                  a.offi + c0 + half * 8);
          lds_u4[halo_u4(hv) + half] = val;
        }
      }
      // weights of the taps of this plane: rows (tap, n), 16 channels each
      for (int e = threadIdx.x; e < 9 * N * 2; e += 256) {
        const int row = e >> 1, half = e & 1;
        const int tap = pz * 9 + row / N, n = row % N;
        lds_u4[CH_PAD_U4 + wrow_u4(row, half)] =
            *reinterpret_cast<const uint4*>(a.W + ((int64_t)tap * N + n) * a.Cin + c0 + half * 8);
      }
      __syncthreads();
#pragma unroll 3
      for (int tt = 0; tt < 9; ++tt) {
        const int tap = pz * 9 + tt;
        const int toff = sgn * ((tap % 3 - 1) + CH_X * ((tap / 3) % 3 - 1 + CH_Y * (tap / 9 - 1)));
        short4_ Bv[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          Bv[nt] = *reinterpret_cast<const short4_*>(ws + wrow_el(tt * N + nt * 16 + ml, kg));
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
          const int v = hb[mt] + toff;
          const short4_ A = *reinterpret_cast<const short4_*>(xs + halo_el(v, v / CH_X) + kg * 4);
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
            acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, Bv[nt], acc[mt][nt], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = (wave * 4 + mt) * 16 + 4 * kg + j;
      const int gx = x0 + q % CT_X, gy = y0 + (q / CT_X) % CT_Y, gz = z0 + q / (CT_X * CT_Y);
      if (gx >= D || gy >= D || gz >= D) continue;
      const int64_t v = sbase + gx + (int64_t)D * (gy + (int64_t)D * gz);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int n = nt * 16 + ml;
        float rv = acc[mt][nt][j] + (a.bias ? a.bias[n] : 0.f);
        if (a.relu && !(rv > 0.f)) rv = 0.f;
        if (a.mask && !(b2f(a.mask[v * a.ldm + a.offm + n]) > 0.f)) rv = 0.f;
        a.out[v * a.ldo + a.offo + n] = f2bf(rv);
      }
    }
}

// Same tiling with plane reuse, for NT <= 2. The halo is staged in LDS. With
// 16 output channels the weight fragments (27 x 16 rows of 32 B per chunk,
// read by every workgroup) come from the caches, so that the LDS holds
// only the halo (20 KB: eight workgroups per CU; 463 -> 385 us per launch at
// 48^3 x 64); with 32 they are staged in LDS next to it (reading them from
// the caches was slower there, 130 -> 159 us). Wave w owns a 16-voxel xy patch (rows 2w, 2w+1 of
// the 8x8 block) through all 4 output planes. For each in-plane tap offset it
// walks the 6 halo planes once: every input fragment it reads from LDS feeds
// the MFMAs of up to 3 output planes (one per z tap), which halves the LDS
// reads of the plain form. The weights are each MFMA's A operand and the
// voxels its B operand (so that a lane's results are four channels of one
// voxel). With 32 output channels each MFMA is gfx950's K = 32 form and
// takes two in-plane taps at once (16 channels each), twice the rate of the
// K = 16 one.
template <int NT, int FLIP>
__global__ __launch_bounds__(256) void k_conv3_zr(ConvArgs a, int ntx, int nty, int ntz, int64_t ntiles,
                                                  int64_t per) {
  extern __shared__ uint4 lds_u4[];
  // LDS: the halo [CH_V][CCH] (rows padded) in CH_PAD_U4 16-byte units, then
  // the weights [27][N][CCH] when staged
  const bf16* xs = reinterpret_cast<const bf16*>(lds_u4);
  constexpr int N = NT * 16;
  constexpr int SG = FLIP ? -1 : 1;
  constexpr bool WLDS = NT >= 2;  // weights staged in LDS
  const int64_t t = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (t >= ntiles) return;  // whole workgroup leaves together
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ml = lane & 15, kg = lane >> 4;
  const int D = a.D;
  int64_t r = t;
  const int tx = (int)(r % ntx);
  r /= ntx;
  const int ty = (int)(r % nty);
  r /= nty;
  const int tz = (int)(r % ntz);
  const int64_t b = r / ntz;
  const int x0 = tx * CT_X, y0 = ty * CT_Y, z0 = tz * CT_Z;
  const int64_t sbase = b * (int64_t)D * D * D;
  const int qa = wave * 16 + ml;  // my A row: xy voxel of the patch
  const int hxy = (qa % CT_X + 1) + CH_X * (qa / CT_X + 1);
  float4_ acc[CT_Z][NT];
#pragma unroll
  for (int z = 0; z < CT_Z; ++z)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[z][nt] = float4_{0.f, 0.f, 0.f, 0.f};
  const int dh = D / 2;  // edge of a half-resolution first input
  const int64_t sbase_h = b * (int64_t)dh * dh * dh;
  for (int c0 = 0; c0 < a.Cin; c0 += CCH) {
    __syncthreads();
    // the chunk's source: the second input, the half-resolution first input,
    // or the first input
    const bool second = a.in2 && c0 >= a.C1, half_res = !second && a.up1;
    for (int e = threadIdx.x; e < CH_V * 2; e += 256) {
      const int hv = e >> 1, half = e & 1;
      const int gx = x0 + hv % CH_X - 1, gy = y0 + (hv / CH_X) % CH_Y - 1, gz = z0 + hv / (CH_X * CH_Y) - 1;
      uint4 val{0u, 0u, 0u, 0u};
      if (gx >= 0 && gx < D && gy >= 0 && gy < D && gz >= 0 && gz < D) {
        const bf16* src;
        if (second)
          src = a.in2 + (sbase + gx + (int64_t)D * (gy + (int64_t)D * gz)) * a.ldi2 + (c0 - a.C1);
        else if (half_res)
          src = a.in + (sbase_h + (gx >> 1) + (int64_t)dh * ((gy >> 1) + (int64_t)dh * (gz >> 1))) * a.ldi + a.offi + c0;
        else
          src = a.in + (sbase + gx + (int64_t)D * (gy + (int64_t)D * gz)) * a.ldi + a.offi + c0;
        val = *reinterpret_cast<const uint4*>(src + half * 8);
      }
      lds_u4[halo_u4(hv) + half] = val;
    }
    if (WLDS)
      for (int e = threadIdx.x; e < 27 * N * 2; e += 256) {
        const int row = e >> 1, half = e & 1;  // row = tap * N + n
        lds_u4[CH_PAD_U4 + wrow_u4(row, half)] =
            *reinterpret_cast<const uint4*>(a.W + (int64_t)row * a.Cin + c0 + half * 8);
      }
    __syncthreads();
    if constexpr (NT == 1) {
      // 16 output channels: one in-plane tap per MFMA (K = 16), the weight
      // fragments read from the caches, those of the next tap issued before
      // this tap's MFMAs. This form keeps about 40 VGPRs (eight waves per
      // SIMD); the K = 32 form below needs 80 and was slower here (254 -> 278
      // us at Cin = 16), faster with 32 output channels.
      auto load_w = [&](int txy, short4_ (&Wt)[3]) {
#pragma unroll
        for (int k = 0; k < 3; ++k)
          Wt[k] = *reinterpret_cast<const short4_*>(a.W + (int64_t)((txy + 9 * k) * N + ml) * a.Cin + c0 + kg * 4);
      };
      short4_ Wt[3], Wn[3];  // z taps dz = -1, 0, 1
      load_w(0, Wn);
#pragma unroll 1
      for (int txy = 0; txy < 9; ++txy) {
        const int dxt = txy % 3 - 1, dyt = txy / 3 - 1;  // the tap's in-plane offsets
        const int hoff = SG * dxt + CH_X * (SG * dyt);
        const int rxy = (hxy + hoff) / CH_X;  // halo row of the tap's voxel in plane 0
#pragma unroll
        for (int k = 0; k < 3; ++k) Wt[k] = Wn[k];
        if (txy + 1 < 9) load_w(txy + 1, Wn);
#pragma unroll
        for (int p = 0; p < CH_Z; ++p) {
          const short4_ Xf = *reinterpret_cast<const short4_*>(
              xs + halo_el(hxy + hoff + CH_X * CH_Y * p, rxy + CH_Y * p) + kg * 4);
#pragma unroll
          for (int z = 0; z < CT_Z; ++z) {
            const int dzin = p - 1 - z;  // input plane offset seen from output plane z
            if (dzin < -1 || dzin > 1) continue;
            acc[z][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Wt[SG * dzin + 1], Xf, acc[z][0], 0, 0, 0);
          }
        }
      }
    } else {
      // Two in-plane taps per MFMA (v_mfma_f32_16x16x32_bf16, K = 32): in step j
      // lane groups kg = 0, 1 take tap 2 j and kg = 2, 3 tap 2 j + 1 (none for
      // j = 4: zeros), channels 8 (kg & 1) .. 8 (kg & 1) + 7 of the chunk, in the
      // weight and the voxel fragment alike. Weight rows come from LDS; those
      // of step j + 1 are read before step j's MFMAs, and step j's six voxel
      // fragments (one per halo plane) before its first MFMA. Every load is issued by every lane
      // (lanes without a tap read tap 8's and zero it), so none sits behind a
      // branch.
      const int hsel = kg & 1;
      auto load_w = [&](int j, bf16x8 (&Wt)[3][NT]) {
        const int tl = 2 * j + (kg >> 1);
        const bool tv = tl < 9;
        const int tc = tv ? tl : 8;
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const int row = (tc + 9 * k) * N + nt * 16 + ml;
            uint4 w = lds_u4[CH_PAD_U4 + wrow_u4(row, hsel)];
            if (!tv) w = uint4{0u, 0u, 0u, 0u};
            Wt[k][nt] = __builtin_bit_cast(bf16x8, w);
          }
      };
      bf16x8 W2[2][3][NT];  // steps j and j + 1 by parity; z taps dz = -1, 0, 1
      load_w(0, W2[0]);
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        bf16x8 (&Wt)[3][NT] = W2[j & 1];
        if (j + 1 < 5) load_w(j + 1, W2[(j + 1) & 1]);
        const int tl = 2 * j + (kg >> 1);  // this lane group's in-plane tap
        const bool tv = tl < 9;
        const int tc = tv ? tl : 8;
        const int dxt = tc % 3 - 1, dyt = tc / 3 - 1;
        const int v0 = hxy + SG * dxt + CH_X * (SG * dyt);  // halo voxel of the tap, plane 0
        // plane p of voxel v0 is voxel v0 + CH_X CH_Y p, in halo row v0 / CH_X + CH_Y p
        const uint4* ap = lds_u4 + halo_u4(v0) + hsel;
        constexpr int PSTEP = 2 * CH_X * CH_Y + CH_Y;  // 16-byte units per halo plane
        bf16x8 Xv[CH_Z];
#pragma unroll
        for (int p = 0; p < CH_Z; ++p) {
          uint4 av = ap[PSTEP * p];
          if (!tv) av = uint4{0u, 0u, 0u, 0u};
          Xv[p] = __builtin_bit_cast(bf16x8, av);
        }
#pragma unroll
        for (int p = 0; p < CH_Z; ++p) {
#pragma unroll
          for (int z = 0; z < CT_Z; ++z) {
            const int dzin = p - 1 - z;  // input plane offset seen from output plane z
            if (dzin < -1 || dzin > 1) continue;
            const int k = SG * dzin + 1;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
              acc[z][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Wt[k][nt], Xv[p], acc[z][nt], 0, 0, 0);
          }
        }
      }
    }
  }
  // The weights are the MFMA's A operand and the voxels its B operand, so
  // lane (ml, kg) holds output channels 4 kg .. 4 kg + 3 (of each 16-channel
  // tile) of voxel qa: one 8-byte store per output plane and tile.
  const int gx = x0 + qa % CT_X, gy = y0 + qa / CT_X;
#pragma unroll
  for (int z = 0; z < CT_Z; ++z) {
    const int gz = z0 + z;
    if (gx >= D || gy >= D || gz >= D) continue;
    const int64_t v = sbase + gx + (int64_t)D * (gy + (int64_t)D * gz);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int n0 = nt * 16 + 4 * kg;
      uint2 mk{0xffffffffu, 0xffffffffu};  // BF16 pairs; all positive where no mask
      if (a.mask) mk = *reinterpret_cast<const uint2*>(a.mask + v * a.ldm + a.offm + n0);
      uint32_t o[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        uint32_t packed = 0;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int j = 2 * h + e;
          float rv = acc[z][nt][j] + (a.bias ? a.bias[n0 + j] : 0.f);
          if (a.relu && !(rv > 0.f)) rv = 0.f;
          const uint32_t mw = h ? mk.y : mk.x;
          if (a.mask && !(b2f((bf16)(e ? mw >> 16 : mw & 0xffffu)) > 0.f)) rv = 0.f;
          packed |= (uint32_t)f2bf(rv) << (16 * e);
        }
        o[h] = packed;
      }
      *reinterpret_cast<uint2*>(a.out + v * a.ldo + a.offo + n0) = uint2{o[0], o[1]};
    }
  }
}

template <int NT, int FLIP>
static void conv3_zr_launch(const ConvArgs& a, hipStream_t s) {
  const int ntx = (a.D + CT_X - 1) / CT_X, nty = (a.D + CT_Y - 1) / CT_Y, ntz = (a.D + CT_Z - 1) / CT_Z;
  const int64_t ntiles = (int64_t)a.B * ntx * nty * ntz;
  const int64_t per = (ntiles + 7) / 8;
  const size_t lds = sizeof(bf16) * (CH_PAD_U4 * 8 + (NT >= 2 ? 27 * NT * 16 * CCH : 0));
  hipLaunchKernelGGL((k_conv3_zr<NT, FLIP>), dim3((unsigned)(8 * per)), dim3(256), lds, s, a, ntx, nty, ntz, ntiles,
                     per);
}

// First layer (4 input channels): one 16-wide K chunk of the MFMA covers
// four taps of 4 channels each (lane group kg takes tap 4c + kg), so the
// halo (8 B per voxel) and all 27 taps of weights sit in LDS at once.
template <int NT>
__global__ __launch_bounds__(256) void k_conv3_c4(ConvArgs a, int ntx, int nty, int ntz, int64_t ntiles,
                                                  int64_t per) {
  constexpr int N = NT * 16;
  __shared__ uint2 xs4[CH_V];
  __shared__ uint2 ws4[27 * N];
  const int64_t t = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (t >= ntiles) return;  // whole workgroup leaves together
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ml = lane & 15, kg = lane >> 4;
  const int D = a.D;
  int64_t r = t;
  const int tx = (int)(r % ntx);
  r /= ntx;
  const int ty = (int)(r % nty);
  r /= nty;
  const int tz = (int)(r % ntz);
  const int64_t b = r / ntz;
  const int x0 = tx * CT_X, y0 = ty * CT_Y, z0 = tz * CT_Z;
  const int64_t sbase = b * (int64_t)D * D * D;
  for (int e = threadIdx.x; e < CH_V; e += 256) {
    const int gx = x0 + e % CH_X - 1, gy = y0 + (e / CH_X) % CH_Y - 1, gz = z0 + e / (CH_X * CH_Y) - 1;
    uint2 val{0u, 0u};
    if (gx >= 0 && gx < D && gy >= 0 && gy < D && gz >= 0 && gz < D)
      val = *reinterpret_cast<const uint2*>(a.in + (sbase + gx + (int64_t)D * (gy + (int64_t)D * gz)) * a.ldi + a.offi);
    xs4[e] = val;
  }
  for (int e = threadIdx.x; e < 27 * N; e += 256) ws4[e] = *reinterpret_cast<const uint2*>(a.W + (int64_t)e * 4);
  __syncthreads();
  int hb[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const int q = (wave * 4 + mt) * 16 + ml;
    hb[mt] = (q % CT_X + 1) + CH_X * ((q / CT_X) % CT_Y + 1 + CH_Y * (q / (CT_X * CT_Y) + 1));
  }
  float4_ acc[4][NT];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = float4_{0.f, 0.f, 0.f, 0.f};
  const int sgn = a.flip ? -1 : 1;
#pragma unroll
  for (int c = 0; c < 7; ++c) {
    const int tap = 4 * c + kg;
    const bool ok = tap < 27;
    const int toff = ok ? sgn * ((tap % 3 - 1) + CH_X * ((tap / 3) % 3 - 1 + CH_Y * (tap / 9 - 1))) : 0;
    short4_ Bv[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
      Bv[nt] = ok ? __builtin_bit_cast(short4_, ws4[tap * N + nt * 16 + ml]) : short4_{0, 0, 0, 0};
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const short4_ A = ok ? __builtin_bit_cast(short4_, xs4[hb[mt] + toff]) : short4_{0, 0, 0, 0};
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Bv[nt], A, acc[mt][nt], 0, 0, 0);
    }
  }
  // weights as the MFMA's A operand, voxels as its B: lane (ml, kg) holds
  // output channels 4 kg .. 4 kg + 3 of voxel (4 wave + mt) 16 + ml, one
  // 8-byte store per M tile
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const int q = (wave * 4 + mt) * 16 + ml;
    const int gx = x0 + q % CT_X, gy = y0 + (q / CT_X) % CT_Y, gz = z0 + q / (CT_X * CT_Y);
    if (gx >= D || gy >= D || gz >= D) continue;
    const int64_t v = sbase + gx + (int64_t)D * (gy + (int64_t)D * gz);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int n0 = nt * 16 + 4 * kg;
      uint2 mk{0xffffffffu, 0xffffffffu};  // BF16 pairs; all positive where no mask
      if (a.mask) mk = *reinterpret_cast<const uint2*>(a.mask + v * a.ldm + a.offm + n0);
      uint32_t o[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        uint32_t packed = 0;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int j = 2 * h + e;
          float rv = acc[mt][nt][j] + (a.bias ? a.bias[n0 + j] : 0.f);
          if (a.relu && !(rv > 0.f)) rv = 0.f;
          const uint32_t mw = h ? mk.y : mk.x;
          if (a.mask && !(b2f((bf16)(e ? mw >> 16 : mw & 0xffffu)) > 0.f)) rv = 0.f;
          packed |= (uint32_t)f2bf(rv) << (16 * e);
        }
        o[h] = packed;
      }
      *reinterpret_cast<uint2*>(a.out + v * a.ldo + a.offo + n0) = uint2{o[0], o[1]};
    }
  }
}

template <int NT>
static void conv3_lds_launch(const ConvArgs& a, hipStream_t s) {
  const int ntx = (a.D + CT_X - 1) / CT_X, nty = (a.D + CT_Y - 1) / CT_Y, ntz = (a.D + CT_Z - 1) / CT_Z;
  const int64_t ntiles = (int64_t)a.B * ntx * nty * ntz;
  const int64_t per = (ntiles + 7) / 8;
  const size_t lds = sizeof(bf16) * (CH_PAD_U4 * 8 + 9 * NT * 16 * CCH);
  hipLaunchKernelGGL(k_conv3_lds<NT>, dim3((unsigned)(8 * per)), dim3(256), lds, s, a, ntx, nty, ntz, ntiles, per);
}

static void conv3(const ConvArgs& a, hipStream_t s) {
  if (a.in2 || a.up1) {
    // two inputs: the z-reuse kernels only
    if (a.Cin % CCH != 0 || (a.in2 && (a.C1 % CCH != 0 || a.C1 <= 0 || a.C1 >= a.Cin)) || (a.up1 && a.D % 2 != 0))
      fatal_combo("conv3 second input");
    switch (a.N / 16) {
      case 1: a.flip ? conv3_zr_launch<1, 1>(a, s) : conv3_zr_launch<1, 0>(a, s); return;
      case 2: a.flip ? conv3_zr_launch<2, 1>(a, s) : conv3_zr_launch<2, 0>(a, s); return;
      default: fatal_combo("conv3 second input: output channels");
    }
  }
  if (a.Cin == 4 && a.N == 16 && a.ldi == 4 && a.offi == 0) {
    const int ntx = (a.D + CT_X - 1) / CT_X, nty = (a.D + CT_Y - 1) / CT_Y, ntz = (a.D + CT_Z - 1) / CT_Z;
    const int64_t ntiles = (int64_t)a.B * ntx * nty * ntz;
    const int64_t per = (ntiles + 7) / 8;
    hipLaunchKernelGGL(k_conv3_c4<1>, dim3((unsigned)(8 * per)), dim3(256), 0, s, a, ntx, nty, ntz, ntiles, per);
    return;
  }
  if (a.Cin % CCH == 0) {
    switch (a.N / 16) {
      case 1: a.flip ? conv3_zr_launch<1, 1>(a, s) : conv3_zr_launch<1, 0>(a, s); return;
      case 2: a.flip ? conv3_zr_launch<2, 1>(a, s) : conv3_zr_launch<2, 0>(a, s); return;
      case 3: conv3_lds_launch<3>(a, s); return;
      case 4: conv3_lds_launch<4>(a, s); return;
      case 6: conv3_lds_launch<6>(a, s); return;
      default: fatal_combo("conv3 output channels");
    }
  }
  const int64_t total = (int64_t)a.B * a.D * a.D * a.D;
  const dim3 gr((unsigned)((total + 127) / 128));
  switch (a.N / 16) {
    case 1: hipLaunchKernelGGL(k_conv3<1>, gr, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_conv3<2>, gr, dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_conv3<3>, gr, dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_conv3<4>, gr, dim3(256), 0, s, a); break;
    case 6: hipLaunchKernelGGL(k_conv3<6>, gr, dim3(256), 0, s, a); break;
    default: fatal_combo("conv3 output channels");
  }
}

// ---------------------------------------------------------------------------
// Weight gradient of a 3x3x3 layer: part[chunk][t][ci][co] =
// sum over the chunk's voxels v of X[v + off(t)][ci] dY[v][co] (FP32), with
// a 32-voxel tile of X (shifted by the tap) and dY staged in LDS.
// ---------------------------------------------------------------------------
constexpr int WG_TILE = 32;
constexpr int WG_CHUNK = 4096;  // voxels per partial

__global__ __launch_bounds__(256) void k_wgrad_part(int B, int D, int Cin, int Cout, const bf16* __restrict__ X,
                                                    int ldx, int offx, const bf16* __restrict__ dY, int ldy,
                                                    int offy, float* __restrict__ part) {
  extern __shared__ float smem[];
  float* Xs = smem;                   // [WG_TILE][Cin]
  float* Ys = smem + WG_TILE * Cin;   // [WG_TILE][Cout]
  const int tap = blockIdx.y;
  const int64_t V = (int64_t)D * D * D, total = (int64_t)B * V;
  const int64_t c0 = (int64_t)blockIdx.x * WG_CHUNK;
  const int no = Cin * Cout;
  const int dx = tap % 3 - 1, dy = (tap / 3) % 3 - 1, dz = tap / 9 - 1;
  float acc[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = 0.f;
  for (int64_t t0 = c0; t0 < c0 + WG_CHUNK && t0 < total; t0 += WG_TILE) {
    __syncthreads();
    for (int e = threadIdx.x; e < WG_TILE * Cin; e += 256) {
      const int r = e / Cin, ci = e - r * Cin;
      const int64_t gv = t0 + r;
      float val = 0.f;
      if (gv < total) {
        const int64_t v = gv % V;
        const int x = (int)(v % D) + dx, y = (int)((v / D) % D) + dy, z = (int)(v / ((int64_t)D * D)) + dz;
        if (x >= 0 && x < D && y >= 0 && y < D && z >= 0 && z < D) {
          const int64_t nb = gv + dx + (int64_t)D * (dy + (int64_t)D * dz);
          val = b2f(X[nb * ldx + offx + ci]);
        }
      }
      Xs[e] = val;
    }
    for (int e = threadIdx.x; e < WG_TILE * Cout; e += 256) {
      const int r = e / Cout, co = e - r * Cout;
      const int64_t gv = t0 + r;
      Ys[e] = gv < total ? b2f(dY[gv * ldy + offy + co]) : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int o = threadIdx.x + 256 * e;
      if (o < no) {
        const int ci = o / Cout, co = o - ci * Cout;
        float s = acc[e];
        for (int r = 0; r < WG_TILE; ++r) s = fmaf(Xs[r * Cin + ci], Ys[r * Cout + co], s);
        acc[e] = s;
      }
    }
  }
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int o = threadIdx.x + 256 * e;
    if (o < no) part[((int64_t)blockIdx.x * 27 + tap) * no + o] = acc[e];
  }
}

// g[i] = sum over chunks of part[chunk][i] (fixed order), i < n.
__global__ void k_sum_chunks(int nchunk, int64_t n, const float* __restrict__ part, float* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * n + i];
  g[i] = s;
}

// Bias gradient: db[co] = sum_v dY[v][co], one workgroup per channel.
__global__ __launch_bounds__(256) void k_bias_grad(int64_t total, int Cout, const bf16* __restrict__ dY, int ldy,
                                                   int offy, float* __restrict__ db) {
  __shared__ float red[256];
  const int co = blockIdx.x;
  float s = 0.f;
  for (int64_t v = threadIdx.x; v < total; v += 256) s += b2f(dY[v * ldy + offy + co]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[co] = red[0];
}

// ---------------------------------------------------------------------------
// Pooling, upsampling, skip gradients (channels last, slices of wider buffers)
// ---------------------------------------------------------------------------
// Eight channels (16 B) per thread; every channel count, stride and slice
// offset here is a multiple of 8.
__device__ inline void ld8(const bf16* p, float f[8]) {
  const uint4 w = *reinterpret_cast<const uint4*>(p);
  const uint32_t u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    f[2 * k] = b2f((bf16)(u[k] & 0xffffu));
    f[2 * k + 1] = b2f((bf16)(u[k] >> 16));
  }
}
__device__ inline void st8(bf16* p, const float f[8]) {
  uint32_t u[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) u[k] = (uint32_t)f2bf(f[2 * k]) | ((uint32_t)f2bf(f[2 * k + 1]) << 16);
  *reinterpret_cast<uint4*>(p) = uint4{u[0], u[1], u[2], u[3]};
}
__device__ inline int64_t child(int D, int x, int y, int z, int k) {
  return (2 * x + (k & 1)) + (int64_t)D * ((2 * y + ((k >> 1) & 1)) + (int64_t)D * (2 * z + (k >> 2)));
}

// out [B][d^3] (row stride ldo) = 2x average pooling of the slice (ldi, offi) of in [B][D^3].
__global__ void k_pool2(int B, int D, int C, const bf16* __restrict__ in, int ldi, int offi, bf16* __restrict__ out,
                        int ldo) {
  const int d = D / 2, G = C / 8;
  const int64_t Vd = (int64_t)d * d * d;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)B * Vd * G) return;
  const int c = (int)(t % G) * 8;
  const int64_t bv = t / G, b = bv / Vd, v = bv % Vd;
  const int x = (int)(v % d), y = (int)((v / d) % d), z = (int)(v / ((int64_t)d * d));
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, f[8];
  for (int k = 0; k < 8; ++k) {
    ld8(in + (b * D * D * D + child(D, x, y, z, k)) * ldi + offi + c, f);
#pragma unroll
    for (int e = 0; e < 8; ++e) s[e] += f[e];
  }
#pragma unroll
  for (int e = 0; e < 8; ++e) s[e] *= 0.125f;
  st8(out + bv * ldo + c, s);
}

// out slice [B][(2d)^3][C] at (ldo, offo) = nearest upsampling of in [B][d^3][C]
__global__ void k_up2(int B, int d, int C, const bf16* __restrict__ in, bf16* __restrict__ out, int ldo, int offo) {
  const int D = 2 * d, G = C / 8;
  const int64_t VD = (int64_t)D * D * D;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)B * VD * G) return;
  const int c = (int)(t % G) * 8;
  const int64_t bv = t / G, b = bv / VD, v = bv % VD;
  const int x = (int)(v % D), y = (int)((v / D) % D), z = (int)(v / ((int64_t)D * D));
  const int64_t iv = (x / 2) + (int64_t)d * ((y / 2) + (int64_t)d * (z / 2));
  *reinterpret_cast<uint4*>(out + bv * ldo + offo + c) =
      *reinterpret_cast<const uint4*>(in + (b * d * d * d + iv) * C + c);
}

// out [B][d^3][C] = (sum over the 8 children of the gradient slice) masked
// by (act > 0) where act is [B][d^3][C].
__global__ void k_up2_bwd(int B, int d, int C, const bf16* __restrict__ g, int ldg, int offg,
                          const bf16* __restrict__ act, bf16* __restrict__ out) {
  const int D = 2 * d, G = C / 8;
  const int64_t Vd = (int64_t)d * d * d;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)B * Vd * G) return;
  const int c = (int)(t % G) * 8;
  const int64_t bv = t / G, b = bv / Vd, v = bv % Vd;
  const int x = (int)(v % d), y = (int)((v / d) % d), z = (int)(v / ((int64_t)d * d));
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, f[8], a[8];
  for (int k = 0; k < 8; ++k) {
    ld8(g + (b * D * D * D + child(D, x, y, z, k)) * ldg + offg + c, f);
#pragma unroll
    for (int e = 0; e < 8; ++e) s[e] += f[e];
  }
  ld8(act + bv * C + c, a);
#pragma unroll
  for (int e = 0; e < 8; ++e)
    if (!(a[e] > 0.f)) s[e] = 0.f;
  st8(out + bv * C + c, s);
}

// Gradient of a skip activation s (= a slice of a concat buffer): the
// decoder's slice gradient plus 1/8 of the pooled gradient of its parent,
// masked by (s > 0). out [B][D^3][C].
__global__ void k_skip_grad(int B, int D, int C, const bf16* __restrict__ gcat, int ldc, int offc,
                            const bf16* __restrict__ gpool, const bf16* __restrict__ s, int lds, int offs,
                            bf16* __restrict__ out) {
  const int d = D / 2, G = C / 8;
  const int64_t VD = (int64_t)D * D * D;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)B * VD * G) return;
  const int c = (int)(t % G) * 8;
  const int64_t bv = t / G, b = bv / VD, v = bv % VD;
  const int x = (int)(v % D), y = (int)((v / D) % D), z = (int)(v / ((int64_t)D * D));
  const int64_t pv = (x / 2) + (int64_t)d * ((y / 2) + (int64_t)d * (z / 2));
  float gc[8], gp[8], sv[8], r[8];
  ld8(gcat + bv * ldc + offc + c, gc);
  ld8(gpool + (b * d * d * d + pv) * C + c, gp);
  ld8(s + bv * lds + offs + c, sv);
#pragma unroll
  for (int e = 0; e < 8; ++e) r[e] = sv[e] > 0.f ? gc[e] + 0.125f * gp[e] : 0.f;
  st8(out + bv * C + c, r);
}

// ---------------------------------------------------------------------------
// 1x1 head (16 -> 2, linear, FP32 output) and its backward
// ---------------------------------------------------------------------------
__global__ void k_head_fwd(int64_t total, const bf16* __restrict__ a, const float* __restrict__ W,
                           const float* __restrict__ b, float* __restrict__ out) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= total) return;
  float o0 = b[0], o1 = b[1];
  for (int ci = 0; ci < 16; ++ci) {
    const float x = b2f(a[v * 16 + ci]);
    o0 = fmaf(x, W[ci * 2 + 0], o0);
    o1 = fmaf(x, W[ci * 2 + 1], o1);
  }
  out[v * 2 + 0] = o0;
  out[v * 2 + 1] = o1;
}

// ga[v][ci] = (sum_co W[ci][co] dout[v][co]) masked by a > 0; partial head
// weight gradients per workgroup: part[blk][0..31] = sum a*dout, [32..33] = sum dout.
__global__ __launch_bounds__(256) void k_head_bwd(int64_t total, const bf16* __restrict__ a,
                                                  const float* __restrict__ W, const float* __restrict__ dout,
                                                  bf16* __restrict__ ga, float* __restrict__ part) {
  __shared__ float red[256];
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float g0 = 0.f, g1 = 0.f;
  float xs[16];
  if (v < total) {
    g0 = dout[v * 2 + 0];
    g1 = dout[v * 2 + 1];
    for (int ci = 0; ci < 16; ++ci) {
      const float x = b2f(a[v * 16 + ci]);
      xs[ci] = x;
      const float g = W[ci * 2] * g0 + W[ci * 2 + 1] * g1;
      ga[v * 16 + ci] = f2bf(x > 0.f ? g : 0.f);
    }
  } else {
    for (int ci = 0; ci < 16; ++ci) xs[ci] = 0.f;
  }
  for (int e = 0; e < 34; ++e) {
    float val;
    if (e < 32) val = xs[e / 2] * ((e & 1) ? g1 : g0);
    else val = (e == 32) ? g0 : g1;
    red[threadIdx.x] = val;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * 34 + e] = red[0];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Loss: per sample num = sum_mask |out - t|^2, den = sum_mask |t|^2;
// dout = mask ? 2 (out - t) / den / B : 0.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_loss_sums(int64_t V, const float* __restrict__ out,
                                                   const float* __restrict__ tgt, const uint8_t* __restrict__ mask,
                                                   float* __restrict__ numden) {
  __shared__ float rn[256], rd[256];
  const int s = blockIdx.x;
  float n = 0.f, d = 0.f;
  for (int64_t v = threadIdx.x; v < V; v += 256) {
    if (!mask[v]) continue;
    const int64_t i = ((int64_t)s * V + v) * 2;
    const float e0 = out[i] - tgt[i], e1 = out[i + 1] - tgt[i + 1];
    n += e0 * e0 + e1 * e1;
    d += tgt[i] * tgt[i] + tgt[i + 1] * tgt[i + 1];
  }
  rn[threadIdx.x] = n;
  rd[threadIdx.x] = d;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      rn[threadIdx.x] += rn[threadIdx.x + w];
      rd[threadIdx.x] += rd[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    numden[2 * s] = rn[0];
    numden[2 * s + 1] = rd[0];
  }
}

__global__ void k_loss_grad(int B, int64_t V, const float* __restrict__ out, const float* __restrict__ tgt,
                            const uint8_t* __restrict__ mask, const float* __restrict__ numden,
                            float* __restrict__ dout) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)B * V) return;
  const int64_t s = t / V, v = t % V;
  const float den = numden[2 * s + 1];
  const float f = (mask[v] && den > 0.f) ? 2.f / den / B : 0.f;
  dout[2 * t] = f * (out[2 * t] - tgt[2 * t]);
  dout[2 * t + 1] = f * (out[2 * t + 1] - tgt[2 * t + 1]);
}

// ---------------------------------------------------------------------------
// Parameters: FP32 master (oracle packing), BF16 working layouts, Adam.
// ---------------------------------------------------------------------------
// Wf[t][co][ci] (forward) and Wb[t][ci][co] (backward data) from W[t][ci][co].
__global__ void k_wpack(int Cin, int Cout, const float* __restrict__ W, bf16* __restrict__ Wf, bf16* __restrict__ Wb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 27LL * Cin * Cout) return;
  const int co = (int)(t % Cout);
  const int64_t r = t / Cout;
  const int ci = (int)(r % Cin), tap = (int)(r / Cin);
  const bf16 w = f2bf(W[t]);
  Wb[t] = w;
  Wf[((int64_t)tap * Cout + co) * Cin + ci] = w;
}

__global__ void k_adam(int64_t n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------
// Glue with the solver: coarse fields [Nc][P] <-> network volumes. The
// unknown (x, y, z) of the nx x ny x nz coarsest grid sits at voxel (x, y, z)
// of the D^3 volume; the rest of the volume is padding (input 0).
// ---------------------------------------------------------------------------
struct Box {
  int nx, ny, nz;
};

__device__ inline int64_t box_index(const Box& b, int D, int64_t v) {
  const int x = (int)(v % D), y = (int)((v / D) % D), z = (int)(v / ((int64_t)D * D));
  if (x >= b.nx || y >= b.ny || z >= b.nz) return -1;
  return x + (int64_t)b.nx * (y + (int64_t)b.ny * z);
}

__device__ inline uint2 pack_in(float a, float b, float c, float d) {
  return uint2{(uint32_t)f2bf(a) | ((uint32_t)f2bf(b) << 16), (uint32_t)f2bf(c) | ((uint32_t)f2bf(d) << 16)};
}

// Sample b < nb of x0 = (Re, Im of f[n][c0 + b] sc[c0 + b], Re, Im of dgn[n]).
template <class S>
__global__ void k_net_input(int P, int c0, int nb, int D, Box bx, const S* __restrict__ f,
                            const double* __restrict__ sc, const float* __restrict__ dgn, bf16* __restrict__ x0) {
  const int64_t V = (int64_t)D * D * D;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nb * V) return;
  const int c = c0 + (int)(t / V);
  const int64_t n = box_index(bx, D, t % V);
  uint2 w{0u, 0u};
  if (n >= 0) {
    const S fv = f[n * P + c];
    const float s = (float)sc[c];
    w = pack_in((float)fv.re * s, (float)fv.im * s, dgn[2 * n], dgn[2 * n + 1]);
  }
  reinterpret_cast<uint2*>(x0)[t] = w;
}

// e[n][c0 + b] = os[c0 + b] (out[b][v][0] + i out[b][v][1]); counts
// non-finite or implausibly large outputs in *bad.
template <class S>
__global__ void k_net_output(int P, int c0, int nb, int D, Box bx, const float* __restrict__ out,
                             const double* __restrict__ os, S* __restrict__ e, int* __restrict__ bad) {
  const int64_t Nc = (int64_t)bx.nx * bx.ny * bx.nz;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= Nc * nb) return;
  const int64_t n = t / nb;
  const int b = (int)(t % nb);
  const int x = (int)(n % bx.nx), y = (int)((n / bx.nx) % bx.ny), z = (int)(n / ((int64_t)bx.nx * bx.ny));
  const int64_t v = (int64_t)b * D * D * D + x + (int64_t)D * (y + (int64_t)D * z);
  const float o0 = out[2 * v], o1 = out[2 * v + 1];
  // targets e / (H^2 rms) are of order one: an output beyond 1e4 in these
  // units is as useless as a non-finite one and is counted with them
  if (!(fabsf(o0) <= 1e4f) || !(fabsf(o1) <= 1e4f)) atomicAdd(bad, 1);
  using E = decltype(e->re);
  e[n * P + c0 + b] = S{(E)(os[c0 + b] * o0), (E)(os[c0 + b] * o1)};
}

// Training pair of column c into pool slot `slot`: input as k_net_input and
// target e / (H^2 rms) (FP32, 0 in the padding).
template <class S>
__global__ void k_capture(int P, int c, int D, Box bx, const S* __restrict__ f, const S* __restrict__ e,
                          const double* __restrict__ sc, double h2inv, const float* __restrict__ dgn, int64_t slot,
                          bf16* __restrict__ xs, float* __restrict__ ts) {
  const int64_t V = (int64_t)D * D * D;
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const int64_t n = box_index(bx, D, v);
  uint2 w{0u, 0u};
  float t0 = 0.f, t1 = 0.f;
  if (n >= 0) {
    const S fv = f[n * P + c], ev = e[n * P + c];
    const float s = (float)sc[c];
    w = pack_in((float)fv.re * s, (float)fv.im * s, dgn[2 * n], dgn[2 * n + 1]);
    t0 = (float)((double)ev.re * sc[c] * h2inv);
    t1 = (float)((double)ev.im * sc[c] * h2inv);
  }
  reinterpret_cast<uint2*>(xs)[slot * V + v] = w;
  ts[2 * (slot * V + v)] = t0;
  ts[2 * (slot * V + v) + 1] = t1;
}

// dgn[n] = H^2 (centre coefficient of the coarsest stencil) as FP32 pairs.
__global__ void k_net_dgn(int64_t N, int NS, const c128* __restrict__ st, double h2, float* __restrict__ dgn) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const c128 a = st[n * NS + NS / 2];
  dgn[2 * n] = (float)(h2 * a.re);
  dgn[2 * n + 1] = (float)(h2 * a.im);
}

// mask[v] = 1 on voxels that hold an unknown.
__global__ void k_net_mask(int D, Box bx, uint8_t* __restrict__ mask) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= (int64_t)D * D * D) return;
  mask[v] = box_index(bx, D, v) >= 0 ? 1 : 0;
}

// sc[c] = 1/rms (0 for a zero column), os[c] = H^2 rms, from ||f_c||^2.
__global__ void k_net_scales(int P, int64_t Nc, double h2, const double* __restrict__ n2, double* __restrict__ sc,
                             double* __restrict__ os) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P) return;
  const double rms = sqrt(n2[c] / (double)Nc);
  sc[c] = rms > 0.0 ? 1.0 / rms : 0.0;
  os[c] = h2 * rms;
}

// Minibatch sample b = pool entry idx[b] with its residual and target turned
// by the unit phase rot[b] = (cos, sin): the exact coarsest solve commutes
// with that rotation, so every phase is a valid training pair.
__global__ void k_gather_samples(int nb, const int* __restrict__ idx, const float* __restrict__ rot, int64_t V,
                                 const bf16* __restrict__ xs, const float* __restrict__ ts, bf16* __restrict__ x0,
                                 float* __restrict__ tgt) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nb * V) return;
  const int b = (int)(t / V);
  const int64_t v = t % V;
  const int64_t src = (int64_t)idx[b] * V + v;
  const float cs = rot[2 * b], sn = rot[2 * b + 1];
  const uint2 w = reinterpret_cast<const uint2*>(xs)[src];
  const float xr = b2f((bf16)(w.x & 0xffffu)), xi = b2f((bf16)(w.x >> 16));
  const float yr = cs * xr - sn * xi, yi = sn * xr + cs * xi;
  reinterpret_cast<uint2*>(x0)[t] = uint2{(uint32_t)f2bf(yr) | ((uint32_t)f2bf(yi) << 16), w.y};
  const float tr = ts[2 * src], ti = ts[2 * src + 1];
  tgt[2 * t] = cs * tr - sn * ti;
  tgt[2 * t + 1] = sn * tr + cs * ti;
}

// loss = (1/B) sum over samples with den > 0 of num / den.
__global__ void k_loss_value(int B, const float* __restrict__ numden, float* __restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float l = 0.f;
  for (int s = 0; s < B; ++s)
    if (numden[2 * s + 1] > 0.f) l += numden[2 * s] / numden[2 * s + 1];
  *loss = l / B;
}

__global__ void k_zero_int(int* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

__global__ void k_f32_to_bf16(int64_t n, const float* __restrict__ a, bf16* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = f2bf(a[i]);
}

__global__ void k_bf16_to_f32(int64_t n, const bf16* __restrict__ a, float* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = b2f(a[i]);
}

static inline dim3 g1(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------
struct Net {
  int D = 0, Bmax = 0;
  int64_t V = 0;
  int64_t np = 0;
  float* p = nullptr;   // FP32 master parameters, packed as the oracle packs them
  float* g = nullptr;   // gradient
  float* am = nullptr;  // Adam moments
  float* av = nullptr;
  int64_t adam_t = 0;
  void* wmem = nullptr;
  bf16* Wf[NLAYER] = {};
  bf16* Wb[NLAYER] = {};
  // activations (channels last, BF16) for Bmax samples
  void* amem = nullptr;
  bf16 *x0 = nullptr, *a1 = nullptr, *c1 = nullptr, *p1 = nullptr, *a2 = nullptr, *c2 = nullptr, *p2 = nullptr,
       *a4 = nullptr, *a5 = nullptr, *a6 = nullptr, *a7 = nullptr, *a8 = nullptr, *a9 = nullptr;
  float* out = nullptr;
  float* numden = nullptr;
  float* lossd = nullptr;
  // backward buffers (allocated on first use)
  void* bmem = nullptr;
  float *dout = nullptr, *tgt = nullptr, *wpart = nullptr, *hpart = nullptr;
  bf16 *g9 = nullptr, *g8 = nullptr, *gc1 = nullptr, *g7 = nullptr, *g6 = nullptr, *gc2 = nullptr, *g5 = nullptr,
       *g4 = nullptr, *gp2 = nullptr, *g3 = nullptr, *g2 = nullptr, *gp1 = nullptr, *g1 = nullptr, *g0 = nullptr;
  int* idx = nullptr;
  float* rot = nullptr;
  float* hist = nullptr;
  int hist_n = 0;
  // binding to a coarsest grid
  bool bound = false;
  Box box{0, 0, 0};
  int64_t Nc = 0;
  double H2 = 1.0;
  Prec pf = P64;
  float* dgn = nullptr;
  uint8_t* mask = nullptr;
  double* n2 = nullptr;  // [Pmax] column norms^2, then scales
  double* sc = nullptr;
  double* os = nullptr;
  c128* part = nullptr;
  c128* Gs = nullptr;
  int Pmax = 0;
  uint64_t scratch_gen = 0;  // bumped whenever the per-column scratch moves
  int* bad = nullptr;
  int* hbad = nullptr;     // pinned
  double* hn2 = nullptr;   // pinned [Pmax]
  // pool of training pairs
  int cap_max = 0, cap_n = 0;
  int64_t cap_seen = 0;
  Box cap_box{0, 0, 0};  // coarsest grid the pool's pairs live on
  bf16* xs = nullptr;
  float* ts = nullptr;
  std::mt19937_64 rng{12345};
};

#define LCHECK(expr)                                                                                   \
  do {                                                                                                 \
    hipError_t e_ = (expr);                                                                            \
    if (e_ != hipSuccess)                                                                              \
      return fail(e_ == hipErrorOutOfMemory ? HELM_ERR_OOM : HELM_ERR_DEVICE, "network: %s: %s", #expr, \
                  hipGetErrorString(e_));                                                              \
  } while (0)

static size_t al(size_t b) { return (b + 255) / 256 * 256; }

int64_t nparams() { return nparams_total(); }

int edge_for(const Coarse& g) {
  const int m = std::max(g.nu[0], std::max(g.nu[1], g.nu[2]));
  return (m + 3) / 4 * 4;
}

static void pack_weights(Net* n, hipStream_t s) {
  for (int l = 0; l < NLAYER; ++l) {
    const int64_t nw = 27LL * L_CIN[l] * L_COUT[l];
    hipLaunchKernelGGL(k_wpack, g1(nw), dim3(256), 0, s, L_CIN[l], L_COUT[l], n->p + layer_off(l), n->Wf[l], n->Wb[l]);
  }
}

helm_status create(int D, int max_batch, uint64_t seed, hipStream_t s, Net** out) {
  *out = nullptr;
  if (D < 4 || D % 4 != 0 || D > 256) return fail(HELM_ERR_INVALID_ARG, "network edge D=%d must be a multiple of 4 in 4..256", D);
  if (max_batch < 1 || max_batch > 1024) return fail(HELM_ERR_INVALID_ARG, "max_batch must be 1..1024");
  Net* n = new Net();
  n->D = D;
  n->Bmax = max_batch;
  n->V = (int64_t)D * D * D;
  n->np = nparams_total();
  auto bail = [&](helm_status st) {
    destroy(n);
    return st;
  };
  const size_t pb = al(4 * (size_t)n->np);
  if (dmalloc(&n->p, 4 * pb) != hipSuccess) return bail(fail(HELM_ERR_OOM, "network parameters"));
  n->g = n->p + pb / 4;
  n->am = n->g + pb / 4;
  n->av = n->am + pb / 4;
  int64_t nw = 0;
  for (int l = 0; l < NLAYER; ++l) nw += al(2 * 27LL * L_CIN[l] * L_COUT[l]);
  if (dmalloc(&n->wmem, 2 * nw) != hipSuccess) return bail(fail(HELM_ERR_OOM, "network weights"));
  char* w = static_cast<char*>(n->wmem);
  for (int l = 0; l < NLAYER; ++l) {
    const size_t b = al(2 * 27LL * L_CIN[l] * L_COUT[l]);
    n->Wf[l] = reinterpret_cast<bf16*>(w);
    n->Wb[l] = reinterpret_cast<bf16*>(w + b);
    w += 2 * b;
  }
  // activations
  const int64_t BV = (int64_t)max_batch * n->V, BV2 = BV / 8, BV4 = BV / 64;
  const size_t sizes[] = {al(2 * BV * 4),   al(2 * BV * 16),  al(2 * BV * 48),  al(2 * BV2 * 16), al(2 * BV2 * 32),
                          al(2 * BV2 * 96), al(2 * BV4 * 32), al(2 * BV4 * 64), al(2 * BV4 * 64), al(2 * BV2 * 32),
                          al(2 * BV2 * 32), al(2 * BV * 16),  al(2 * BV * 16),  al(4 * BV * 2),   al(8 * (size_t)max_batch),
                          al(4)};
  size_t tot = 0;
  for (size_t b : sizes) tot += b;
  if (dmalloc(&n->amem, tot) != hipSuccess) return bail(fail(HELM_ERR_OOM, "network activations (%zu bytes)", tot));
  char* a = static_cast<char*>(n->amem);
  void** slots[] = {(void**)&n->x0, (void**)&n->a1, (void**)&n->c1, (void**)&n->p1, (void**)&n->a2, (void**)&n->c2,
                    (void**)&n->p2, (void**)&n->a4, (void**)&n->a5, (void**)&n->a6, (void**)&n->a7, (void**)&n->a8,
                    (void**)&n->a9, (void**)&n->out, (void**)&n->numden, (void**)&n->lossd};
  for (size_t k = 0; k < sizeof(sizes) / sizeof(sizes[0]); ++k) {
    *slots[k] = a;
    a += sizes[k];
  }
  if (hipHostMalloc(&n->hbad, sizeof(int)) != hipSuccess) return bail(fail(HELM_ERR_OOM, "pinned host memory"));
  // He-scaled initial weights, zero biases
  std::vector<float> h(n->np, 0.f);
  std::mt19937_64 rng(seed);
  std::normal_distribution<float> nd(0.f, 1.f);
  for (int l = 0; l < NLAYER; ++l) {
    const float sd = std::sqrt(2.f / (27.f * L_CIN[l]));
    const int64_t o = layer_off(l);
    for (int64_t k = 0; k < 27LL * L_CIN[l] * L_COUT[l]; ++k) h[o + k] = sd * nd(rng);
  }
  for (int k = 0; k < 32; ++k) h[n->np - 34 + k] = 0.25f * nd(rng);
  helm_status st = set_params(n, h.data(), s);
  if (st != HELM_OK) return bail(st);
  *out = n;
  return HELM_OK;
}

void destroy(Net* n) {
  if (!n) return;
  hipDeviceSynchronize();
  hipFree(n->p);
  hipFree(n->wmem);
  hipFree(n->amem);
  hipFree(n->bmem);
  hipFree(n->idx);
  hipFree(n->rot);
  hipFree(n->hist);
  hipFree(n->dgn);
  hipFree(n->mask);
  hipFree(n->n2);
  hipFree(n->part);
  hipFree(n->xs);
  hipFree(n->ts);
  if (n->hbad) hipHostFree(n->hbad);
  if (n->hn2) hipHostFree(n->hn2);
  delete n;
}

helm_status set_params(Net* n, const float* host, hipStream_t s) {
  for (int64_t k = 0; k < n->np; ++k)
    if (!std::isfinite(host[k])) return fail(HELM_ERR_NONFINITE, "network parameter %lld is not finite", (long long)k);
  LCHECK(hipMemcpyAsync(n->p, host, 4 * n->np, hipMemcpyHostToDevice, s));
  LCHECK(hipMemsetAsync(n->am, 0, 4 * n->np, s));
  LCHECK(hipMemsetAsync(n->av, 0, 4 * n->np, s));
  n->adam_t = 0;
  pack_weights(n, s);
  LCHECK(hipStreamSynchronize(s));
  return HELM_OK;
}

helm_status get_params(Net* n, float* host, hipStream_t s) {
  LCHECK(hipMemcpyAsync(host, n->p, 4 * n->np, hipMemcpyDeviceToHost, s));
  LCHECK(hipStreamSynchronize(s));
  return HELM_OK;
}

// Training checkpoint: parameters, Adam first and second moments (3 np FP32
// values) and the step count.
helm_status get_state(Net* n, float* host, int64_t* step, hipStream_t s) {
  LCHECK(hipMemcpyAsync(host, n->p, 4 * n->np, hipMemcpyDeviceToHost, s));
  LCHECK(hipMemcpyAsync(host + n->np, n->am, 4 * n->np, hipMemcpyDeviceToHost, s));
  LCHECK(hipMemcpyAsync(host + 2 * n->np, n->av, 4 * n->np, hipMemcpyDeviceToHost, s));
  LCHECK(hipStreamSynchronize(s));
  *step = n->adam_t;
  return HELM_OK;
}

helm_status set_state(Net* n, const float* host, int64_t step, hipStream_t s) {
  if (step < 0) return fail(HELM_ERR_INVALID_ARG, "Adam step count must be >= 0");
  for (int64_t k = 0; k < 3 * n->np; ++k)
    if (!std::isfinite(host[k])) return fail(HELM_ERR_NONFINITE, "training state entry %lld is not finite", (long long)k);
  for (int64_t k = 2 * n->np; k < 3 * n->np; ++k)
    if (host[k] < 0.f) return fail(HELM_ERR_INVALID_ARG, "Adam second moment %lld is negative", (long long)(k - 2 * n->np));
  LCHECK(hipMemcpyAsync(n->p, host, 4 * n->np, hipMemcpyHostToDevice, s));
  LCHECK(hipMemcpyAsync(n->am, host + n->np, 4 * n->np, hipMemcpyHostToDevice, s));
  LCHECK(hipMemcpyAsync(n->av, host + 2 * n->np, 4 * n->np, hipMemcpyHostToDevice, s));
  n->adam_t = step;
  pack_weights(n, s);
  LCHECK(hipStreamSynchronize(s));
  return HELM_OK;
}

size_t blob_bytes() { return 16 + 4 * (size_t)nparams_total(); }

helm_status write_blob(Net* n, void* blob, hipStream_t s) {
  char* b = static_cast<char*>(blob);
  std::memcpy(b, "HNET", 4);
  const uint32_t ver = 1;
  const int64_t np = n->np;
  std::memcpy(b + 4, &ver, 4);
  std::memcpy(b + 8, &np, 8);
  return get_params(n, reinterpret_cast<float*>(b + 16), s);
}

helm_status read_blob(const void* blob, size_t bytes, float* params) {
  const char* b = static_cast<const char*>(blob);
  if (!blob || bytes < 16 || std::memcmp(b, "HNET", 4) != 0) return fail(HELM_ERR_INVALID_ARG, "network blob: bad header");
  uint32_t ver;
  int64_t np;
  std::memcpy(&ver, b + 4, 4);
  std::memcpy(&np, b + 8, 8);
  if (ver != 1 || np != nparams_total() || bytes != blob_bytes())
    return fail(HELM_ERR_INVALID_ARG, "network blob: version %u, %lld parameters, %zu bytes (expected 1, %lld, %zu)", ver,
                (long long)np, bytes, (long long)nparams_total(), blob_bytes());
  std::memcpy(params, b + 16, 4 * (size_t)np);
  return HELM_OK;
}

// ---- passes -----------------------------------------------------------------
static void conv_fwd(Net* n, int l, int B, int D, const bf16* in, int ldi, int offi, bf16* out, int ldo, int offo,
                     hipStream_t s) {
  ConvArgs a{};
  a.B = B;
  a.D = D;
  a.Cin = L_CIN[l];
  a.N = L_COUT[l];
  a.in = in;
  a.ldi = ldi;
  a.offi = offi;
  a.W = n->Wf[l];
  a.bias = n->p + layer_off(l) + 27LL * L_CIN[l] * L_COUT[l];
  a.out = out;
  a.ldo = ldo;
  a.offo = offo;
  a.flip = 0;
  a.relu = 1;
  conv3(a, s);
}

// gx = (adjoint of layer l's convolution) dy, optionally masked by act > 0.
static void conv_bwd_data(Net* n, int l, int B, int D, const bf16* dy, bf16* gx, int ldx, const bf16* act,
                          hipStream_t s) {
  ConvArgs a{};
  a.B = B;
  a.D = D;
  a.Cin = L_COUT[l];
  a.N = L_CIN[l];
  a.in = dy;
  a.ldi = L_COUT[l];
  a.offi = 0;
  a.W = n->Wb[l];
  a.bias = nullptr;
  a.out = gx;
  a.ldo = ldx;
  a.offo = 0;
  a.flip = 1;
  a.relu = 0;
  a.mask = act;
  a.ldm = L_CIN[l];
  a.offm = 0;
  conv3(a, s);
}

static void conv_bwd_weight(Net* n, int l, int B, int D, const bf16* x, int ldx, int offx, const bf16* dy,
                            hipStream_t s) {
  const int Cin = L_CIN[l], Cout = L_COUT[l];
  const int64_t total = (int64_t)B * D * D * D;
  const int nchunk = (int)((total + WG_CHUNK - 1) / WG_CHUNK);
  const size_t lds = sizeof(float) * WG_TILE * (Cin + Cout);
  hipLaunchKernelGGL(k_wgrad_part, dim3(nchunk, 27), dim3(256), lds, s, B, D, Cin, Cout, x, ldx, offx, dy, Cout, 0,
                     n->wpart);
  const int64_t nw = 27LL * Cin * Cout;
  float* gW = n->g + layer_off(l);
  hipLaunchKernelGGL(k_sum_chunks, g1(nw), dim3(256), 0, s, nchunk, nw, (const float*)n->wpart, gW);
  hipLaunchKernelGGL(k_bias_grad, dim3(Cout), dim3(256), 0, s, total, Cout, dy, Cout, 0, gW + nw);
}

// Decoder layer l reading the upsampled coarser activations `up` (C1
// channels, row stride ldu, grid edge D / 2) and the skip activations `skip`
// (row stride lds) as one input of C1 + (Cin - C1) channels, in that order.
static void conv_fwd_up(Net* n, int l, int B, int D, const bf16* up, int ldu, int C1, const bf16* skip, int lds,
                        bf16* out, int ldo, hipStream_t s) {
  ConvArgs a{};
  a.B = B;
  a.D = D;
  a.Cin = L_CIN[l];
  a.N = L_COUT[l];
  a.in = up;
  a.ldi = ldu;
  a.offi = 0;
  a.up1 = 1;
  a.in2 = skip;
  a.ldi2 = lds;
  a.C1 = C1;
  a.W = n->Wf[l];
  a.bias = n->p + layer_off(l) + 27LL * L_CIN[l] * L_COUT[l];
  a.out = out;
  a.ldo = ldo;
  a.offo = 0;
  a.flip = 0;
  a.relu = 1;
  conv3(a, s);
}

// The forward pass. With `concat` (training, whose backward pass reads the
// decoder inputs as stored activations) the skip outputs s1, s2 go into
// slices of c1, c2 and the upsampled activations are copied beside them;
// without it (inference) s1 and s2 are stored densely in c1, c2 and the two
// decoder layers that take them read the coarser activations and the skip
// outputs directly. Both forms give every convolution the same values in
// the same channel order, so their outputs are equal bit for bit.
static void run_forward(Net* n, int B, hipStream_t s, bool concat) {
  const int D = n->D, d2 = D / 2, d4 = D / 4;
  const int64_t BV = (int64_t)B * n->V;
  if (!concat) {
    conv_fwd(n, 0, B, D, n->x0, 4, 0, n->a1, 16, 0, s);
    conv_fwd(n, 1, B, D, n->a1, 16, 0, n->c1, 16, 0, s);  // s1, dense
    hipLaunchKernelGGL(k_pool2, g1(BV / 8 * 2), dim3(256), 0, s, B, D, 16, (const bf16*)n->c1, 16, 0, n->p1, 16);
    conv_fwd(n, 2, B, d2, n->p1, 16, 0, n->a2, 32, 0, s);
    conv_fwd(n, 3, B, d2, n->a2, 32, 0, n->c2, 32, 0, s);  // s2, dense
    hipLaunchKernelGGL(k_pool2, g1(BV / 64 * 4), dim3(256), 0, s, B, d2, 32, (const bf16*)n->c2, 32, 0, n->p2, 32);
    conv_fwd(n, 4, B, d4, n->p2, 32, 0, n->a4, 64, 0, s);
    conv_fwd(n, 5, B, d4, n->a4, 64, 0, n->a5, 64, 0, s);
    conv_fwd_up(n, 6, B, d2, n->a5, 64, 64, n->c2, 32, n->a6, 32, s);
    conv_fwd(n, 7, B, d2, n->a6, 32, 0, n->a7, 32, 0, s);
    conv_fwd_up(n, 8, B, D, n->a7, 32, 32, n->c1, 16, n->a8, 16, s);
    conv_fwd(n, 9, B, D, n->a8, 16, 0, n->a9, 16, 0, s);
    hipLaunchKernelGGL(k_head_fwd, g1(BV), dim3(256), 0, s, BV, (const bf16*)n->a9,
                       (const float*)(n->p + n->np - 34), (const float*)(n->p + n->np - 2), n->out);
    return;
  }
  conv_fwd(n, 0, B, D, n->x0, 4, 0, n->a1, 16, 0, s);
  conv_fwd(n, 1, B, D, n->a1, 16, 0, n->c1, 48, 32, s);  // s1 -> second slice of c1
  hipLaunchKernelGGL(k_pool2, g1(BV / 8 * 2), dim3(256), 0, s, B, D, 16, (const bf16*)n->c1, 48, 32, n->p1, 16);
  conv_fwd(n, 2, B, d2, n->p1, 16, 0, n->a2, 32, 0, s);
  conv_fwd(n, 3, B, d2, n->a2, 32, 0, n->c2, 96, 64, s);  // s2 -> second slice of c2
  hipLaunchKernelGGL(k_pool2, g1(BV / 64 * 4), dim3(256), 0, s, B, d2, 32, (const bf16*)n->c2, 96, 64, n->p2, 32);
  conv_fwd(n, 4, B, d4, n->p2, 32, 0, n->a4, 64, 0, s);
  conv_fwd(n, 5, B, d4, n->a4, 64, 0, n->a5, 64, 0, s);
  hipLaunchKernelGGL(k_up2, g1(BV / 8 * 8), dim3(256), 0, s, B, d4, 64, (const bf16*)n->a5, n->c2, 96, 0);
  conv_fwd(n, 6, B, d2, n->c2, 96, 0, n->a6, 32, 0, s);
  conv_fwd(n, 7, B, d2, n->a6, 32, 0, n->a7, 32, 0, s);
  hipLaunchKernelGGL(k_up2, g1(BV * 4), dim3(256), 0, s, B, d2, 32, (const bf16*)n->a7, n->c1, 48, 0);
  conv_fwd(n, 8, B, D, n->c1, 48, 0, n->a8, 16, 0, s);
  conv_fwd(n, 9, B, D, n->a8, 16, 0, n->a9, 16, 0, s);
  hipLaunchKernelGGL(k_head_fwd, g1(BV), dim3(256), 0, s, BV, (const bf16*)n->a9, (const float*)(n->p + n->np - 34),
                     (const float*)(n->p + n->np - 2), n->out);
}

static helm_status ensure_backward(Net* n) {
  if (n->bmem) return HELM_OK;
  const int64_t BV = (int64_t)n->Bmax * n->V, BV2 = BV / 8, BV4 = BV / 64;
  int64_t wp = 0;
  const int64_t vox[3] = {BV, BV2, BV4};
  const int lev[NLAYER] = {0, 0, 1, 1, 2, 2, 1, 1, 0, 0};
  for (int l = 0; l < NLAYER; ++l) {
    const int64_t nch = (vox[lev[l]] + WG_CHUNK - 1) / WG_CHUNK;
    wp = std::max<int64_t>(wp, nch * 27 * L_CIN[l] * L_COUT[l]);
  }
  const int64_t hblk = (BV + 255) / 256;
  const size_t sizes[] = {al(4 * BV * 2),    al(4 * BV * 2),    al(4 * (size_t)wp), al(4 * hblk * 34),
                          al(2 * BV * 16),   al(2 * BV * 16),   al(2 * BV * 48),    al(2 * BV2 * 32),
                          al(2 * BV2 * 32),  al(2 * BV2 * 96),  al(2 * BV4 * 64),   al(2 * BV4 * 64),
                          al(2 * BV4 * 32),  al(2 * BV2 * 32),  al(2 * BV2 * 32),   al(2 * BV2 * 16),
                          al(2 * BV * 16),   al(2 * BV * 16)};
  size_t tot = 0;
  for (size_t b : sizes) tot += b;
  if (dmalloc(&n->bmem, tot) != hipSuccess) return fail(HELM_ERR_OOM, "network gradients (%zu bytes)", tot);
  char* a = static_cast<char*>(n->bmem);
  void** slots[] = {(void**)&n->dout, (void**)&n->tgt, (void**)&n->wpart, (void**)&n->hpart, (void**)&n->g9,
                    (void**)&n->g8,   (void**)&n->gc1, (void**)&n->g7,    (void**)&n->g6,    (void**)&n->gc2,
                    (void**)&n->g5,   (void**)&n->g4,  (void**)&n->gp2,   (void**)&n->g3,    (void**)&n->g2,
                    (void**)&n->gp1,  (void**)&n->g1,  (void**)&n->g0};
  for (size_t k = 0; k < sizeof(sizes) / sizeof(sizes[0]); ++k) {
    *slots[k] = a;
    a += sizes[k];
  }
  return HELM_OK;
}

// Loss of the forward output against n->tgt on `mask`, gradient into n->g.
static void run_loss_backward(Net* n, int B, const uint8_t* mask, float* loss_dst, hipStream_t s) {
  const int D = n->D, d2 = D / 2, d4 = D / 4;
  const int64_t BV = (int64_t)B * n->V;
  hipLaunchKernelGGL(k_loss_sums, dim3(B), dim3(256), 0, s, n->V, (const float*)n->out, (const float*)n->tgt, mask,
                     n->numden);
  hipLaunchKernelGGL(k_loss_value, dim3(1), dim3(64), 0, s, B, (const float*)n->numden, loss_dst);
  hipLaunchKernelGGL(k_loss_grad, g1(BV), dim3(256), 0, s, B, n->V, (const float*)n->out, (const float*)n->tgt, mask,
                     (const float*)n->numden, n->dout);
  // head
  const int64_t hblk = (BV + 255) / 256;
  hipLaunchKernelGGL(k_head_bwd, dim3((unsigned)hblk), dim3(256), 0, s, BV, (const bf16*)n->a9,
                     (const float*)(n->p + n->np - 34), (const float*)n->dout, n->g9, n->hpart);
  hipLaunchKernelGGL(k_sum_chunks, dim3(1), dim3(64), 0, s, (int)hblk, (int64_t)34, (const float*)n->hpart,
                     n->g + n->np - 34);
  // decoder, full resolution
  conv_bwd_weight(n, 9, B, D, n->a8, 16, 0, n->g9, s);
  conv_bwd_data(n, 9, B, D, n->g9, n->g8, 16, n->a8, s);
  conv_bwd_weight(n, 8, B, D, n->c1, 48, 0, n->g8, s);
  conv_bwd_data(n, 8, B, D, n->g8, n->gc1, 48, nullptr, s);
  hipLaunchKernelGGL(k_up2_bwd, g1(BV / 8 * 4), dim3(256), 0, s, B, d2, 32, (const bf16*)n->gc1, 48, 0,
                     (const bf16*)n->a7, n->g7);
  // decoder, half resolution
  conv_bwd_weight(n, 7, B, d2, n->a6, 32, 0, n->g7, s);
  conv_bwd_data(n, 7, B, d2, n->g7, n->g6, 32, n->a6, s);
  conv_bwd_weight(n, 6, B, d2, n->c2, 96, 0, n->g6, s);
  conv_bwd_data(n, 6, B, d2, n->g6, n->gc2, 96, nullptr, s);
  hipLaunchKernelGGL(k_up2_bwd, g1(BV / 64 * 8), dim3(256), 0, s, B, d4, 64, (const bf16*)n->gc2, 96, 0,
                     (const bf16*)n->a5, n->g5);
  // bottom
  conv_bwd_weight(n, 5, B, d4, n->a4, 64, 0, n->g5, s);
  conv_bwd_data(n, 5, B, d4, n->g5, n->g4, 64, n->a4, s);
  conv_bwd_weight(n, 4, B, d4, n->p2, 32, 0, n->g4, s);
  conv_bwd_data(n, 4, B, d4, n->g4, n->gp2, 32, nullptr, s);
  // encoder, half resolution: s2 feeds the pool and the skip
  hipLaunchKernelGGL(k_skip_grad, g1(BV / 8 * 4), dim3(256), 0, s, B, d2, 32, (const bf16*)n->gc2, 96, 64,
                     (const bf16*)n->gp2, (const bf16*)n->c2, 96, 64, n->g3);
  conv_bwd_weight(n, 3, B, d2, n->a2, 32, 0, n->g3, s);
  conv_bwd_data(n, 3, B, d2, n->g3, n->g2, 32, n->a2, s);
  conv_bwd_weight(n, 2, B, d2, n->p1, 16, 0, n->g2, s);
  conv_bwd_data(n, 2, B, d2, n->g2, n->gp1, 16, nullptr, s);
  // encoder, full resolution: s1 feeds the pool and the skip
  hipLaunchKernelGGL(k_skip_grad, g1(BV * 2), dim3(256), 0, s, B, D, 16, (const bf16*)n->gc1, 48, 32,
                     (const bf16*)n->gp1, (const bf16*)n->c1, 48, 32, n->g1);
  conv_bwd_weight(n, 1, B, D, n->a1, 16, 0, n->g1, s);
  conv_bwd_data(n, 1, B, D, n->g1, n->g0, 16, n->a1, s);
  conv_bwd_weight(n, 0, B, D, n->x0, 4, 0, n->g0, s);
}

// HELM_NET_CONCAT=1 makes the inference passes take the training form of the
// forward pass (the check that both forms agree)
static bool concat_forward() {
  const char* e = std::getenv("HELM_NET_CONCAT");
  return e && e[0] == '1';
}

helm_status forward(Net* n, int B, const float* x, float* out, hipStream_t s) {
  if (B < 1 || B > n->Bmax) return fail(HELM_ERR_INVALID_ARG, "batch %d outside 1..%d", B, n->Bmax);
  if (!x || !out) return fail(HELM_ERR_INVALID_ARG, "null buffer");
  const int64_t BV = (int64_t)B * n->V;
  hipLaunchKernelGGL(k_f32_to_bf16, g1(BV * 4), dim3(256), 0, s, BV * 4, x, n->x0);
  run_forward(n, B, s, concat_forward());
  LCHECK(hipMemcpyAsync(out, n->out, 8 * BV, hipMemcpyDeviceToDevice, s));
  LCHECK(hipStreamSynchronize(s));
  LCHECK(hipGetLastError());
  return HELM_OK;
}

helm_status loss_grad(Net* n, int B, const float* x, const float* target, const uint8_t* mask, float* grad,
                      double* loss, hipStream_t s) {
  if (B < 1 || B > n->Bmax) return fail(HELM_ERR_INVALID_ARG, "batch %d outside 1..%d", B, n->Bmax);
  if (!x || !target || !mask || !grad) return fail(HELM_ERR_INVALID_ARG, "null buffer");
  helm_status st = ensure_backward(n);
  if (st != HELM_OK) return st;
  const int64_t BV = (int64_t)B * n->V;
  hipLaunchKernelGGL(k_f32_to_bf16, g1(BV * 4), dim3(256), 0, s, BV * 4, x, n->x0);
  LCHECK(hipMemcpyAsync(n->tgt, target, 8 * BV, hipMemcpyDeviceToDevice, s));
  run_forward(n, B, s, true);
  run_loss_backward(n, B, mask, n->lossd, s);
  LCHECK(hipMemcpyAsync(grad, n->g, 4 * n->np, hipMemcpyDeviceToDevice, s));
  float lf = 0.f;
  LCHECK(hipMemcpyAsync(&lf, n->lossd, 4, hipMemcpyDeviceToHost, s));
  LCHECK(hipStreamSynchronize(s));
  LCHECK(hipGetLastError());
  if (loss) *loss = lf;
  return HELM_OK;
}

// ---- solver glue --------------------------------------------------------------
helm_status bind(Net* n, const Coarse& g, hipStream_t s) {
  if (edge_for(g) != n->D)
    return fail(HELM_ERR_INVALID_ARG, "network edge %d does not fit a %dx%dx%d coarsest grid (needs %d)", n->D, g.nu[0],
                g.nu[1], g.nu[2], edge_for(g));
  if (g.p != P64 && g.p != P32) return fail(HELM_ERR_UNSUPPORTED, "coarsest fields must be FP64 or FP32 complex");
  n->box = Box{g.nu[0], g.nu[1], g.nu[2]};
  n->Nc = (int64_t)g.nu[0] * g.nu[1] * g.nu[2];
  n->H2 = g.H2;
  n->pf = g.p;
  hipFree(n->dgn);
  hipFree(n->mask);
  n->dgn = nullptr;
  n->mask = nullptr;
  LCHECK(dmalloc(&n->dgn, 8 * n->Nc));
  LCHECK(dmalloc(&n->mask, n->V));
  hipLaunchKernelGGL(k_net_dgn, g1(n->Nc), dim3(256), 0, s, n->Nc, 27, g.st, g.H2, n->dgn);
  hipLaunchKernelGGL(k_net_mask, g1(n->V), dim3(256), 0, s, n->D, n->box, n->mask);
  LCHECK(hipStreamSynchronize(s));
  n->bound = true;
  return HELM_OK;
}

static helm_status ensure_cols(Net* n, int P) {
  if (n->Pmax >= P) return HELM_OK;
  hipFree(n->n2);
  hipFree(n->part);
  if (n->hn2) hipHostFree(n->hn2);
  n->n2 = nullptr;
  n->part = nullptr;
  n->hn2 = nullptr;
  n->Pmax = 0;
  LCHECK(dmalloc(&n->n2, 3 * 8 * (size_t)P + 256));
  n->sc = n->n2 + P;
  n->os = n->sc + P;
  LCHECK(dmalloc(&n->part, 16 * (size_t)(gram_part_elems(P) + P)));
  n->Gs = n->part + gram_part_elems(P);
  n->bad = reinterpret_cast<int*>(n->os + P);
  LCHECK(hipHostMalloc(&n->hn2, 8 * (size_t)P));
  n->Pmax = P;
  ++n->scratch_gen;
  return HELM_OK;
}

static void column_scales(Net* n, int P, const void* f, hipStream_t s) {
  launch_colnorm2(n->pf, n->Nc, P, P, f, n->part, n->Gs, n->n2, s);
  hipLaunchKernelGGL(k_net_scales, g1(P), dim3(256), 0, s, P, n->Nc, n->H2, (const double*)n->n2, n->sc, n->os);
}

template <class S>
static void apply_t(Net* n, int P, const S* f, S* out, hipStream_t s) {
  for (int c0 = 0; c0 < P; c0 += n->Bmax) {
    const int nb = std::min(n->Bmax, P - c0);
    hipLaunchKernelGGL(k_net_input<S>, g1((int64_t)nb * n->V), dim3(256), 0, s, P, c0, nb, n->D, n->box, f,
                       (const double*)n->sc, (const float*)n->dgn, n->x0);
    run_forward(n, nb, s, concat_forward());
    hipLaunchKernelGGL(k_net_output<S>, g1(n->Nc * nb), dim3(256), 0, s, P, c0, nb, n->D, n->box,
                       (const float*)n->out, (const double*)n->os, out, n->bad);
  }
}

helm_status prepare(Net* n, int P) {
  if (!n->bound) return fail(HELM_ERR_INVALID_ARG, "network is not bound to a coarsest grid");
  return ensure_cols(n, P);
}

void apply_async(Net* n, int P, const void* f, void* out, hipStream_t s) {
  column_scales(n, P, f, s);
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, s, n->bad);
  if (n->pf == P64)
    apply_t(n, P, static_cast<const c128*>(f), static_cast<c128*>(out), s);
  else
    apply_t(n, P, static_cast<const c64*>(f), static_cast<c64*>(out), s);
}

uint64_t scratch_gen(const Net* n) { return n->scratch_gen; }

int bad_count(Net* n, hipStream_t s) {
  if (!n->bad) return 0;
  if (hipMemcpyAsync(n->hbad, n->bad, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return -1;
  if (hipStreamSynchronize(s) != hipSuccess) return -1;
  return *n->hbad;
}

bool apply(Net* n, int P, const void* f, void* out, hipStream_t s) {
  if (!n->bound || ensure_cols(n, P) != HELM_OK) return false;
  apply_async(n, P, f, out, s);
  return bad_count(n, s) == 0;
}

helm_status capture_begin(Net* n, int max_pairs) {
  if (!n->bound) return fail(HELM_ERR_INVALID_ARG, "network is not bound to a coarsest grid");
  if (max_pairs < 1 || max_pairs > 1 << 20) return fail(HELM_ERR_INVALID_ARG, "max_pairs must be 1..2^20");
  hipFree(n->xs);
  hipFree(n->ts);
  n->xs = nullptr;
  n->ts = nullptr;
  n->cap_max = n->cap_n = 0;
  n->cap_seen = 0;
  LCHECK(dmalloc(&n->xs, 8 * n->V * (size_t)max_pairs));
  LCHECK(dmalloc(&n->ts, 8 * n->V * (size_t)max_pairs));
  n->cap_max = max_pairs;
  n->cap_box = n->box;
  return HELM_OK;
}

helm_status capture_continue(Net* n, const Coarse& g, hipStream_t s) {
  if (n->cap_max < 1) return fail(HELM_ERR_INVALID_ARG, "no pair pool to continue (start one with max_pairs > 0)");
  helm_status st = bind(n, g, s);
  if (st != HELM_OK) return st;
  if (n->box.nx != n->cap_box.nx || n->box.ny != n->cap_box.ny || n->box.nz != n->cap_box.nz)
    return fail(HELM_ERR_INVALID_ARG, "the pool holds %dx%dx%d coarsest grids, this handle has %dx%dx%d",
                n->cap_box.nx, n->cap_box.ny, n->cap_box.nz, n->box.nx, n->box.ny, n->box.nz);
  return HELM_OK;
}

template <class S>
static void capture_t(Net* n, int P, const S* f, const S* e, hipStream_t s) {
  for (int c = 0; c < P; ++c) {
    const double v = n->hn2[c];
    if (!(v > 0.0) || !std::isfinite(v)) continue;  // padding, converged or broken column
    int64_t slot;
    if (n->cap_n < n->cap_max) {
      slot = n->cap_n++;
    } else {
      std::uniform_int_distribution<int64_t> u(0, n->cap_seen);
      slot = u(n->rng);
    }
    ++n->cap_seen;
    if (slot >= n->cap_max) continue;
    hipLaunchKernelGGL(k_capture<S>, g1(n->V), dim3(256), 0, s, P, c, n->D, n->box, f, e, (const double*)n->sc,
                       1.0 / n->H2, (const float*)n->dgn, slot, n->xs, n->ts);
  }
}

void capture(Net* n, int P, const void* f, const void* e, hipStream_t s) {
  if (!n->bound || !n->cap_max || ensure_cols(n, P) != HELM_OK) return;
  column_scales(n, P, f, s);
  if (hipMemcpyAsync(n->hn2, n->n2, 8 * (size_t)P, hipMemcpyDeviceToHost, s) != hipSuccess) return;
  if (hipStreamSynchronize(s) != hipSuccess) return;
  if (n->pf == P64)
    capture_t(n, P, static_cast<const c128*>(f), static_cast<const c128*>(e), s);
  else
    capture_t(n, P, static_cast<const c64*>(f), static_cast<const c64*>(e), s);
}

int64_t pairs(const Net* n) { return n->cap_n; }

helm_status pool_read(Net* n, int64_t i, float* x, float* t, hipStream_t s) {
  if (i < 0 || i >= n->cap_n) return fail(HELM_ERR_INVALID_ARG, "pool index %lld outside 0..%d", (long long)i, n->cap_n - 1);
  if (!x || !t) return fail(HELM_ERR_INVALID_ARG, "null buffer");
  hipLaunchKernelGGL(k_bf16_to_f32, g1(4 * n->V), dim3(256), 0, s, 4 * n->V, (const bf16*)(n->xs + 4 * n->V * i), x);
  LCHECK(hipMemcpyAsync(t, n->ts + 2 * n->V * i, 8 * n->V, hipMemcpyDeviceToDevice, s));
  LCHECK(hipStreamSynchronize(s));
  return HELM_OK;
}

// One Adam step (Kingma & Ba, beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected
// moments) on the FP32 master weights from the gradient in n->g, then the
// BF16 working copies.
static void adam_update(Net* n, double lr, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  ++n->adam_t;
  const float c1 = 1.f - std::pow(b1, (float)n->adam_t), c2 = 1.f - std::pow(b2, (float)n->adam_t);
  hipLaunchKernelGGL(k_adam, g1(n->np), dim3(256), 0, s, n->np, n->p, (const float*)n->g, n->am, n->av, (float)lr, b1,
                     b2, eps, c1, c2);
  pack_weights(n, s);
}

helm_status train_step(Net* n, int B, const float* x, const float* target, const uint8_t* mask, double lr,
                       double* loss, hipStream_t s) {
  if (B < 1 || B > n->Bmax) return fail(HELM_ERR_INVALID_ARG, "batch %d outside 1..%d", B, n->Bmax);
  if (!x || !target || !mask) return fail(HELM_ERR_INVALID_ARG, "null buffer");
  if (!(lr > 0.0)) return fail(HELM_ERR_INVALID_ARG, "lr must be > 0");
  helm_status st = ensure_backward(n);
  if (st != HELM_OK) return st;
  const int64_t BV = (int64_t)B * n->V;
  hipLaunchKernelGGL(k_f32_to_bf16, g1(BV * 4), dim3(256), 0, s, BV * 4, x, n->x0);
  LCHECK(hipMemcpyAsync(n->tgt, target, 8 * BV, hipMemcpyDeviceToDevice, s));
  run_forward(n, B, s, true);
  run_loss_backward(n, B, mask, n->lossd, s);
  adam_update(n, lr, s);
  float lf = 0.f;
  LCHECK(hipMemcpyAsync(&lf, n->lossd, 4, hipMemcpyDeviceToHost, s));
  LCHECK(hipStreamSynchronize(s));
  LCHECK(hipGetLastError());
  if (loss) *loss = lf;
  return HELM_OK;
}

helm_status train(Net* n, int steps, int batch, double lr, uint64_t seed, double* hist, hipStream_t s) {
  if (steps < 1 || batch < 1 || batch > n->Bmax || !(lr > 0.0))
    return fail(HELM_ERR_INVALID_ARG, "steps >= 1, batch 1..%d and lr > 0 are required", n->Bmax);
  if (n->cap_n < 1) return fail(HELM_ERR_INVALID_ARG, "no training pairs captured");
  helm_status st = ensure_backward(n);
  if (st != HELM_OK) return st;
  hipFree(n->idx);
  hipFree(n->rot);
  hipFree(n->hist);
  n->idx = nullptr;
  n->rot = nullptr;
  n->hist = nullptr;
  LCHECK(dmalloc(&n->idx, 4 * (size_t)steps * batch));
  LCHECK(dmalloc(&n->rot, 8 * (size_t)steps * batch));
  LCHECK(dmalloc(&n->hist, 4 * (size_t)steps));
  std::vector<int> idx((size_t)steps * batch);
  std::vector<float> rot(2 * idx.size());
  std::mt19937_64 rng(seed);
  std::uniform_int_distribution<int> u(0, n->cap_n - 1);
  std::uniform_real_distribution<double> ph(0.0, 2.0 * M_PI);
  for (size_t k = 0; k < idx.size(); ++k) {
    idx[k] = u(rng);
    const double a = ph(rng);
    rot[2 * k] = (float)std::cos(a);
    rot[2 * k + 1] = (float)std::sin(a);
  }
  LCHECK(hipMemcpyAsync(n->idx, idx.data(), 4 * idx.size(), hipMemcpyHostToDevice, s));
  LCHECK(hipMemcpyAsync(n->rot, rot.data(), 4 * rot.size(), hipMemcpyHostToDevice, s));
  const int64_t BV = (int64_t)batch * n->V;
  for (int k = 0; k < steps; ++k) {
    hipLaunchKernelGGL(k_gather_samples, g1(BV), dim3(256), 0, s, batch, (const int*)(n->idx + (size_t)k * batch),
                       (const float*)(n->rot + (size_t)2 * k * batch), n->V, (const bf16*)n->xs, (const float*)n->ts,
                       n->x0, n->tgt);
    run_forward(n, batch, s, true);
    run_loss_backward(n, batch, n->mask, n->hist + k, s);
    adam_update(n, lr, s);
  }
  std::vector<float> h(steps);
  LCHECK(hipMemcpyAsync(h.data(), n->hist, 4 * (size_t)steps, hipMemcpyDeviceToHost, s));
  LCHECK(hipStreamSynchronize(s));
  LCHECK(hipGetLastError());
  if (hist)
    for (int k = 0; k < steps; ++k) hist[k] = h[k];
  return HELM_OK;
}

}  // namespace learned
}  // namespace helm
