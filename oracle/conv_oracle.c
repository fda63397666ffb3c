/*
 * conv_oracle.c -- plain FP64 CPU oracle of the learned coarsest-grid
 * correction network (test infrastructure only; see helm_oracle.h).
 *
 * The network is not part of the paper: the paper names a stationary inexact
 * solver of the coarsest grid as future work (end of section 5.3 and the
 * conclusions); this network is that solver's learned form. Every routine
 * here is the plain definition:
 *   - 3x3x3 convolution with zero padding on a D^3 volume, channels last:
 *       y[v][co] = b[co] + sum_t sum_ci x[v + off(t)][ci] W[t][ci][co],
 *     off(t) = (t%3 - 1, (t/3)%3 - 1, t/9 - 1) in (x, y, z), x fastest;
 *   - its adjoints with respect to x (backward data) and W, b (backward
 *     weights);
 *   - 2x average pooling, nearest 2x upsampling and their adjoints;
 *   - ReLU;
 *   - the U-Net composition, its loss and full gradient.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

static inline long vox(int D, int x, int y, int z) { return (long)x + (long)D * ((long)y + (long)D * z); }

void orc_conv3d_fwd(int B, int D, int Cin, int Cout, const double* x, const double* W, const double* b,
                    int relu, double* y) {
  const long V = (long)D * D * D;
#pragma omp parallel for schedule(static)
  for (long bv = 0; bv < (long)B * V; ++bv) {
    const long bb = bv / V, v = bv % V;
    const int X = (int)(v % D), Y = (int)((v / D) % D), Z = (int)(v / ((long)D * D));
    for (int co = 0; co < Cout; ++co) {
      double acc = b ? b[co] : 0.0;
      for (int t = 0; t < 27; ++t) {
        const int xx = X + t % 3 - 1, yy = Y + (t / 3) % 3 - 1, zz = Z + t / 9 - 1;
        if (xx < 0 || xx >= D || yy < 0 || yy >= D || zz < 0 || zz >= D) continue;
        const double* xi = x + (bb * V + vox(D, xx, yy, zz)) * Cin;
        for (int ci = 0; ci < Cin; ++ci) acc += xi[ci] * W[((long)t * Cin + ci) * Cout + co];
      }
      y[bv * Cout + co] = relu && acc < 0.0 ? 0.0 : acc;
    }
  }
}

/* dx = adjoint of x -> conv(x) (no bias, no ReLU) applied to dy. */
void orc_conv3d_bwd_data(int B, int D, int Cin, int Cout, const double* dy, const double* W, double* dx) {
  const long V = (long)D * D * D;
#pragma omp parallel for schedule(static)
  for (long bv = 0; bv < (long)B * V; ++bv) {
    const long bb = bv / V, v = bv % V;
    const int X = (int)(v % D), Y = (int)((v / D) % D), Z = (int)(v / ((long)D * D));
    for (int ci = 0; ci < Cin; ++ci) {
      double acc = 0.0;
      for (int t = 0; t < 27; ++t) {
        /* output voxel u with u + off(t) = v */
        const int xx = X - (t % 3 - 1), yy = Y - ((t / 3) % 3 - 1), zz = Z - (t / 9 - 1);
        if (xx < 0 || xx >= D || yy < 0 || yy >= D || zz < 0 || zz >= D) continue;
        const double* g = dy + (bb * V + vox(D, xx, yy, zz)) * Cout;
        for (int co = 0; co < Cout; ++co) acc += g[co] * W[((long)t * Cin + ci) * Cout + co];
      }
      dx[bv * Cin + ci] = acc;
    }
  }
}

void orc_conv3d_bwd_weight(int B, int D, int Cin, int Cout, const double* x, const double* dy, double* dW,
                           double* db) {
  const long V = (long)D * D * D;
#pragma omp parallel for schedule(static)
  for (int t = 0; t < 27; ++t)
    for (int ci = 0; ci < Cin; ++ci)
      for (int co = 0; co < Cout; ++co) {
        double acc = 0.0;
        for (long bv = 0; bv < (long)B * V; ++bv) {
          const long bb = bv / V, v = bv % V;
          const int X = (int)(v % D), Y = (int)((v / D) % D), Z = (int)(v / ((long)D * D));
          const int xx = X + t % 3 - 1, yy = Y + (t / 3) % 3 - 1, zz = Z + t / 9 - 1;
          if (xx < 0 || xx >= D || yy < 0 || yy >= D || zz < 0 || zz >= D) continue;
          acc += x[(bb * V + vox(D, xx, yy, zz)) * Cin + ci] * dy[bv * Cout + co];
        }
        dW[((long)t * Cin + ci) * Cout + co] = acc;
      }
  if (db)
    for (int co = 0; co < Cout; ++co) {
      double acc = 0.0;
      for (long bv = 0; bv < (long)B * V; ++bv) acc += dy[bv * Cout + co];
      db[co] = acc;
    }
}

/* 1x1x1 convolution (the head): y[v][co] = b[co] + sum_ci x[v][ci] W[ci][co]. */
void orc_conv1_fwd(long n, int Cin, int Cout, const double* x, const double* W, const double* b, double* y) {
  for (long v = 0; v < n; ++v)
    for (int co = 0; co < Cout; ++co) {
      double acc = b ? b[co] : 0.0;
      for (int ci = 0; ci < Cin; ++ci) acc += x[v * Cin + ci] * W[ci * Cout + co];
      y[v * Cout + co] = acc;
    }
}

/* 2x average pooling (D even) and nearest 2x upsampling, channels last. */
void orc_avgpool2(int B, int D, int C, const double* x, double* y) {
  const int d = D / 2;
  for (int bb = 0; bb < B; ++bb)
    for (int z = 0; z < d; ++z)
      for (int yy = 0; yy < d; ++yy)
        for (int xx = 0; xx < d; ++xx)
          for (int c = 0; c < C; ++c) {
            double s = 0.0;
            for (int k = 0; k < 8; ++k)
              s += x[((long)bb * D * D * D + vox(D, 2 * xx + (k & 1), 2 * yy + ((k >> 1) & 1), 2 * z + (k >> 2))) * C + c];
            y[((long)bb * d * d * d + vox(d, xx, yy, z)) * C + c] = 0.125 * s;
          }
}

void orc_upsample2(int B, int d, int C, const double* x, double* y) {
  const int D = 2 * d;
  for (int bb = 0; bb < B; ++bb)
    for (int z = 0; z < D; ++z)
      for (int yy = 0; yy < D; ++yy)
        for (int xx = 0; xx < D; ++xx)
          for (int c = 0; c < C; ++c)
            y[((long)bb * D * D * D + vox(D, xx, yy, z)) * C + c] =
                x[((long)bb * d * d * d + vox(d, xx / 2, yy / 2, z / 2)) * C + c];
}

/* ---------------------------------------------------------------------------
 * The U-Net (3 levels, 16/32/64 channels, skip connections by concatenation)
 * on one D^3 volume per sample, D % 4 == 0. Parameters are packed in layer
 * order: for each 3x3x3 layer W[27][Cin][Cout] then b[Cout]; the 1x1 head
 * W[16][2], b[2]. Layer table (Cin, Cout):
 *   0: 4->16, 1: 16->16 (skip s1), [pool]
 *   2: 16->32, 3: 32->32 (skip s2), [pool]
 *   4: 32->64, 5: 64->64, [up] concat(up, s2)
 *   6: 96->32, 7: 32->32, [up] concat(up, s1)
 *   8: 48->16, 9: 16->16, head 16->2 (linear).
 * ------------------------------------------------------------------------- */
static const int L_CIN[10] = {4, 16, 16, 32, 32, 64, 96, 32, 48, 16};
static const int L_COUT[10] = {16, 16, 32, 32, 64, 64, 32, 32, 16, 16};

long orc_unet_nparams(void) {
  long n = 0;
  for (int l = 0; l < 10; ++l) n += 27L * L_CIN[l] * L_COUT[l] + L_COUT[l];
  return n + 16 * 2 + 2;
}

static void layer_ptr(const double* p, int l, const double** W, const double** b) {
  long o = 0;
  for (int k = 0; k < l; ++k) o += 27L * L_CIN[k] * L_COUT[k] + L_COUT[k];
  *W = p + o;
  *b = p + o + 27L * L_CIN[l] * L_COUT[l];
}

typedef struct {
  double *a0, *a1, *p1, *a2, *a3, *p2, *a4, *a5, *c2, *a6, *a7, *c1, *a8, *a9, *out;
} unet_acts;

static void acts_alloc(unet_acts* A, int B, int D) {
  const long V = (long)B * D * D * D, V2 = V / 8, V4 = V / 64;
  A->a0 = NULL;
  A->a1 = calloc(V * 16, 8);
  A->p1 = calloc(V2 * 16, 8);
  A->a2 = calloc(V2 * 32, 8);
  A->a3 = calloc(V2 * 32, 8);
  A->p2 = calloc(V4 * 32, 8);
  A->a4 = calloc(V4 * 64, 8);
  A->a5 = calloc(V4 * 64, 8);
  A->c2 = calloc(V2 * 96, 8);
  A->a6 = calloc(V2 * 32, 8);
  A->a7 = calloc(V2 * 32, 8);
  A->c1 = calloc(V * 48, 8);
  A->a8 = calloc(V * 16, 8);
  A->a9 = calloc(V * 16, 8);
  A->out = calloc(V * 2, 8);
}

static void acts_free(unet_acts* A) {
  free(A->a1); free(A->p1); free(A->a2); free(A->a3); free(A->p2); free(A->a4); free(A->a5);
  free(A->c2); free(A->a6); free(A->a7); free(A->c1); free(A->a8); free(A->a9); free(A->out);
}

/* dst[v][off + c] = src[v][c] for a channel slice of a wider buffer. */
static void put_slice(long n, int Cs, const double* src, int Cd, int off, double* dst) {
  for (long v = 0; v < n; ++v)
    for (int c = 0; c < Cs; ++c) dst[v * Cd + off + c] = src[v * Cs + c];
}
static void get_slice(long n, int Cd, int off, const double* src, int Cs, double* dst) {
  for (long v = 0; v < n; ++v)
    for (int c = 0; c < Cs; ++c) dst[v * Cs + c] = src[v * Cd + off + c];
}

static void unet_forward_acts(int B, int D, const double* p, const double* x, unet_acts* A) {
  const long V = (long)B * D * D * D, V2 = V / 8;
  const int d2 = D / 2, d4 = D / 4;
  const double *W, *b;
  double* up2 = calloc(V2 * 64, 8);
  double* up1 = calloc(V * 32, 8);
  layer_ptr(p, 0, &W, &b); orc_conv3d_fwd(B, D, 4, 16, x, W, b, 1, A->a0 = A->a1);
  double* s1 = calloc(V * 16, 8);
  layer_ptr(p, 1, &W, &b); orc_conv3d_fwd(B, D, 16, 16, A->a1, W, b, 1, s1);
  orc_avgpool2(B, D, 16, s1, A->p1);
  layer_ptr(p, 2, &W, &b); orc_conv3d_fwd(B, d2, 16, 32, A->p1, W, b, 1, A->a2);
  layer_ptr(p, 3, &W, &b); orc_conv3d_fwd(B, d2, 32, 32, A->a2, W, b, 1, A->a3);
  orc_avgpool2(B, d2, 32, A->a3, A->p2);
  layer_ptr(p, 4, &W, &b); orc_conv3d_fwd(B, d4, 32, 64, A->p2, W, b, 1, A->a4);
  layer_ptr(p, 5, &W, &b); orc_conv3d_fwd(B, d4, 64, 64, A->a4, W, b, 1, A->a5);
  orc_upsample2(B, d4, 64, A->a5, up2);
  put_slice(V2, 64, up2, 96, 0, A->c2);
  put_slice(V2, 32, A->a3, 96, 64, A->c2);
  layer_ptr(p, 6, &W, &b); orc_conv3d_fwd(B, d2, 96, 32, A->c2, W, b, 1, A->a6);
  layer_ptr(p, 7, &W, &b); orc_conv3d_fwd(B, d2, 32, 32, A->a6, W, b, 1, A->a7);
  orc_upsample2(B, d2, 32, A->a7, up1);
  put_slice(V, 32, up1, 48, 0, A->c1);
  put_slice(V, 16, s1, 48, 32, A->c1);
  layer_ptr(p, 8, &W, &b); orc_conv3d_fwd(B, D, 48, 16, A->c1, W, b, 1, A->a8);
  layer_ptr(p, 9, &W, &b); orc_conv3d_fwd(B, D, 16, 16, A->a8, W, b, 1, A->a9);
  orc_conv1_fwd(V, 16, 2, A->a9, p + orc_unet_nparams() - 34, p + orc_unet_nparams() - 2, A->out);
  free(up2);
  free(up1);
  free(s1);
}

/* out[B][D^3][2] = network(x[B][D^3][4]). */
void orc_unet_forward(int B, int D, const double* p, const double* x, double* out) {
  unet_acts A;
  acts_alloc(&A, B, D);
  unet_forward_acts(B, D, p, x, &A);
  memcpy(out, A.out, sizeof(double) * (long)B * D * D * D * 2);
  acts_free(&A);
}

/* Loss = (1/B) sum_s ||out_s - t_s||^2 / ||t_s||^2 over the voxels where
 * mask != 0 (the unknowns of the coarsest grid inside the padded volume), and
 * its gradient with respect to every parameter. Returns the loss. */
static void relu_mask(long n, const double* a, double* g) {
  for (long i = 0; i < n; ++i)
    if (!(a[i] > 0.0)) g[i] = 0.0;
}

double orc_unet_loss_grad(int B, int D, const double* p, const double* x, const double* target,
                          const double* mask, double* grad) {
  const long V = (long)B * D * D * D, Vs = (long)D * D * D, V2 = V / 8, V4 = V / 64;
  const int d2 = D / 2, d4 = D / 4;
  unet_acts A;
  acts_alloc(&A, B, D);
  unet_forward_acts(B, D, p, x, &A);
  /* loss and dL/dout */
  double loss = 0.0;
  double* g_out = calloc(V * 2, 8);
  for (int s = 0; s < B; ++s) {
    double num = 0.0, den = 0.0;
    for (long v = 0; v < Vs; ++v) {
      const long i = (long)s * Vs + v;
      if (mask && mask[v] == 0.0) continue;
      for (int c = 0; c < 2; ++c) {
        const double e = A.out[i * 2 + c] - target[i * 2 + c];
        num += e * e;
        den += target[i * 2 + c] * target[i * 2 + c];
      }
    }
    if (den == 0.0) continue;
    loss += num / den / B;
    for (long v = 0; v < Vs; ++v) {
      const long i = (long)s * Vs + v;
      if (mask && mask[v] == 0.0) continue;
      for (int c = 0; c < 2; ++c) g_out[i * 2 + c] = 2.0 * (A.out[i * 2 + c] - target[i * 2 + c]) / den / B;
    }
  }
  memset(grad, 0, sizeof(double) * orc_unet_nparams());
  const long np = orc_unet_nparams();
  /* head */
  double* g9 = calloc(V * 16, 8);
  {
    const double* Wh = p + np - 34;
    double* gWh = grad + np - 34;
    double* gbh = grad + np - 2;
    for (long v = 0; v < V; ++v)
      for (int co = 0; co < 2; ++co) {
        gbh[co] += g_out[v * 2 + co];
        for (int ci = 0; ci < 16; ++ci) {
          gWh[ci * 2 + co] += A.a9[v * 16 + ci] * g_out[v * 2 + co];
          g9[v * 16 + ci] += Wh[ci * 2 + co] * g_out[v * 2 + co];
        }
      }
  }
#define LGRAD(l, Bn, Dn, cin, cout, xin, gy, gx)                                   \
  do {                                                                             \
    const double *W_, *b_;                                                         \
    layer_ptr(p, l, &W_, &b_);                                                     \
    double *gW_ = (double*)(grad + (W_ - p)), *gb_ = (double*)(grad + (b_ - p));  \
    orc_conv3d_bwd_weight(Bn, Dn, cin, cout, xin, gy, gW_, gb_);                   \
    if (gx) orc_conv3d_bwd_data(Bn, Dn, cin, cout, gy, W_, gx);                    \
  } while (0)
  /* layer 9: a9 = relu(conv(a8)) */
  relu_mask(V * 16, A.a9, g9);
  double* g8 = calloc(V * 16, 8);
  LGRAD(9, B, D, 16, 16, A.a8, g9, g8);
  relu_mask(V * 16, A.a8, g8);
  double* gc1 = calloc(V * 48, 8);
  LGRAD(8, B, D, 48, 16, A.c1, g8, gc1);
  /* c1 = [up(a7), s1]: split */
  double* gup1 = calloc(V * 32, 8);
  double* gs1 = calloc(V * 16, 8);
  get_slice(V, 48, 0, gc1, 32, gup1);
  get_slice(V, 48, 32, gc1, 16, gs1);
  double* g7 = calloc(V2 * 32, 8); /* adjoint of upsampling: sum over children */
  for (int bb = 0; bb < B; ++bb)
    for (int z = 0; z < D; ++z)
      for (int y = 0; y < D; ++y)
        for (int xx = 0; xx < D; ++xx)
          for (int c = 0; c < 32; ++c)
            g7[((long)bb * d2 * d2 * d2 + vox(d2, xx / 2, y / 2, z / 2)) * 32 + c] +=
                gup1[((long)bb * Vs + vox(D, xx, y, z)) * 32 + c];
  relu_mask(V2 * 32, A.a7, g7);
  double* g6 = calloc(V2 * 32, 8);
  LGRAD(7, B, d2, 32, 32, A.a6, g7, g6);
  relu_mask(V2 * 32, A.a6, g6);
  double* gc2 = calloc(V2 * 96, 8);
  LGRAD(6, B, d2, 96, 32, A.c2, g6, gc2);
  double* gup2 = calloc(V2 * 64, 8);
  double* gs2 = calloc(V2 * 32, 8);
  get_slice(V2, 96, 0, gc2, 64, gup2);
  get_slice(V2, 96, 64, gc2, 32, gs2);
  double* g5 = calloc(V4 * 64, 8);
  for (int bb = 0; bb < B; ++bb)
    for (int z = 0; z < d2; ++z)
      for (int y = 0; y < d2; ++y)
        for (int xx = 0; xx < d2; ++xx)
          for (int c = 0; c < 64; ++c)
            g5[((long)bb * d4 * d4 * d4 + vox(d4, xx / 2, y / 2, z / 2)) * 64 + c] +=
                gup2[((long)bb * d2 * d2 * d2 + vox(d2, xx, y, z)) * 64 + c];
  relu_mask(V4 * 64, A.a5, g5);
  double* g4 = calloc(V4 * 64, 8);
  LGRAD(5, B, d4, 64, 64, A.a4, g5, g4);
  relu_mask(V4 * 64, A.a4, g4);
  double* gp2 = calloc(V4 * 32, 8);
  LGRAD(4, B, d4, 32, 64, A.p2, g4, gp2);
  /* a3 feeds the pool and the skip s2 */
  double* g3 = calloc(V2 * 32, 8);
  for (int bb = 0; bb < B; ++bb)
    for (int z = 0; z < d2; ++z)
      for (int y = 0; y < d2; ++y)
        for (int xx = 0; xx < d2; ++xx)
          for (int c = 0; c < 32; ++c) {
            const long i = ((long)bb * d2 * d2 * d2 + vox(d2, xx, y, z)) * 32 + c;
            g3[i] = gs2[i] + 0.125 * gp2[((long)bb * d4 * d4 * d4 + vox(d4, xx / 2, y / 2, z / 2)) * 32 + c];
          }
  relu_mask(V2 * 32, A.a3, g3);
  double* g2 = calloc(V2 * 32, 8);
  LGRAD(3, B, d2, 32, 32, A.a2, g3, g2);
  relu_mask(V2 * 32, A.a2, g2);
  double* gp1 = calloc(V2 * 16, 8);
  LGRAD(2, B, d2, 16, 32, A.p1, g2, gp1);
  /* s1 feeds the pool and the skip (layer 1 output); recompute s1 = relu(conv(a1)) */
  double* s1 = calloc(V * 16, 8);
  {
    const double *W_, *b_;
    layer_ptr(p, 1, &W_, &b_);
    orc_conv3d_fwd(B, D, 16, 16, A.a1, W_, b_, 1, s1);
  }
  double* g1 = calloc(V * 16, 8);
  for (int bb = 0; bb < B; ++bb)
    for (int z = 0; z < D; ++z)
      for (int y = 0; y < D; ++y)
        for (int xx = 0; xx < D; ++xx)
          for (int c = 0; c < 16; ++c) {
            const long i = ((long)bb * Vs + vox(D, xx, y, z)) * 16 + c;
            g1[i] = gs1[i] + 0.125 * gp1[((long)bb * d2 * d2 * d2 + vox(d2, xx / 2, y / 2, z / 2)) * 16 + c];
          }
  relu_mask(V * 16, s1, g1);
  double* g0 = calloc(V * 16, 8);
  LGRAD(1, B, D, 16, 16, A.a1, g1, g0);
  relu_mask(V * 16, A.a1, g0);
  LGRAD(0, B, D, 4, 16, x, g0, (double*)NULL);
#undef LGRAD
  free(g_out); free(g9); free(g8); free(gc1); free(gup1); free(gs1); free(g7); free(g6); free(gc2);
  free(gup2); free(gs2); free(g5); free(g4); free(gp2); free(g3); free(g2); free(gp1); free(s1);
  free(g1); free(g0);
  acts_free(&A);
  return loss;
}
