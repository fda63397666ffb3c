/*
 * helm_oracle.c -- plain FP64 CPU oracle (test infrastructure only; see the
 * header for what each routine follows in the paper). Written for clarity:
 * no blocking, fusion or reordering beyond the definitions. OpenMP only
 * splits independent loops over grid points or right-hand sides.
 */
#include "helm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int64_t og_npts(const og_grid* g) {
  return (int64_t)g->nu[0] * g->nu[1] * g->nu[2];
}

void og_coarsen(const og_grid* f, og_grid* c) {
  c->dim = f->dim;
  for (int a = 0; a < 3; ++a) {
    if (a < f->dim) {
      c->nu[a] = (f->nu[a] + 1) / 2 - 1; /* n cells -> n/2 cells */
      c->h[a] = 2.0 * f->h[a];
    } else {
      c->nu[a] = 1;
      c->h[a] = f->h[a];
    }
  }
}

static inline int64_t gidx(const og_grid* g, int x, int y, int z) {
  return (int64_t)x + (int64_t)g->nu[0] * ((int64_t)y + (int64_t)g->nu[1] * z);
}

static inline void gcoord(const og_grid* g, int64_t i, int* x, int* y, int* z) {
  *x = (int)(i % g->nu[0]);
  int64_t r = i / g->nu[0];
  *y = (int)(r % g->nu[1]);
  *z = (int)(r / g->nu[1]);
}

static inline int inside(const og_grid* g, int x, int y, int z) {
  return x >= 0 && x < g->nu[0] && y >= 0 && y < g->nu[1] && z >= 0 && z < g->nu[2];
}

static inline int ozlo(const og_grid* g) { return g->dim == 3 ? -1 : 0; }
static inline int ozhi(const og_grid* g) { return g->dim == 3 ? 1 : 0; }
static inline int sidx(int ox, int oy, int oz) { return (ox + 1) + 3 * (oy + 1) + 9 * (oz + 1); }

/* ---------------------------------------------------------------------------
 * Operator (eq:helm / eq:LinearSystem): second-order differences per axis.
 * ------------------------------------------------------------------------- */
static inline ozc fine_diag(const og_grid* g, double m, double gam, double omega, double beta) {
  double lap = 0.0;
  for (int a = 0; a < g->dim; ++a) lap += 2.0 / (g->h[a] * g->h[a]);
  return lap - omega * omega * m * (1.0 - I * (gam + beta));
}

void orc_apply_fine(const og_grid* g, const double* m, const double* gamma,
                    double omega, double beta, int nrhs, const ozc* u, ozc* out) {
  const int64_t N = og_npts(g);
  for (int s = 0; s < nrhs; ++s) {
    const ozc* us = u + (int64_t)s * N;
    ozc* os = out + (int64_t)s * N;
#pragma omp parallel for schedule(static) if (N > 32768)
    for (int64_t i = 0; i < N; ++i) {
      int x, y, z;
      gcoord(g, i, &x, &y, &z);
      int c[3] = {x, y, z};
      ozc acc = fine_diag(g, m[i], gamma[i], omega, beta) * us[i];
      for (int a = 0; a < g->dim; ++a) {
        double w = 1.0 / (g->h[a] * g->h[a]);
        for (int sgn = -1; sgn <= 1; sgn += 2) {
          int d[3] = {c[0], c[1], c[2]};
          d[a] += sgn;
          if (inside(g, d[0], d[1], d[2])) acc -= w * us[gidx(g, d[0], d[1], d[2])];
        }
      }
      os[i] = acc;
    }
  }
}

void orc_fine_stencil(const og_grid* g, const double* m, const double* gamma,
                      double omega, double beta, ozc* st) {
  const int64_t N = og_npts(g);
#pragma omp parallel for schedule(static) if (N > 32768)
  for (int64_t i = 0; i < N; ++i) {
    int x, y, z;
    gcoord(g, i, &x, &y, &z);
    ozc* si = st + i * 27;
    for (int k = 0; k < 27; ++k) si[k] = 0;
    si[sidx(0, 0, 0)] = fine_diag(g, m[i], gamma[i], omega, beta);
    int c[3] = {x, y, z};
    for (int a = 0; a < g->dim; ++a) {
      double w = 1.0 / (g->h[a] * g->h[a]);
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        int o[3] = {0, 0, 0};
        o[a] = sgn;
        if (inside(g, c[0] + o[0], c[1] + o[1], c[2] + o[2])) si[sidx(o[0], o[1], o[2])] = -w;
      }
    }
  }
}

void orc_apply_stencil(const og_grid* g, const ozc* st, int nrhs, const ozc* u, ozc* out) {
  const int64_t N = og_npts(g);
  for (int s = 0; s < nrhs; ++s) {
    const ozc* us = u + (int64_t)s * N;
    ozc* os = out + (int64_t)s * N;
#pragma omp parallel for schedule(static) if (N > 8192)
    for (int64_t i = 0; i < N; ++i) {
      int x, y, z;
      gcoord(g, i, &x, &y, &z);
      ozc acc = 0;
      for (int oz = ozlo(g); oz <= ozhi(g); ++oz)
        for (int oy = -1; oy <= 1; ++oy)
          for (int ox = -1; ox <= 1; ++ox)
            if (inside(g, x + ox, y + oy, z + oz))
              acc += st[i * 27 + sidx(ox, oy, oz)] * us[gidx(g, x + ox, y + oy, z + oz)];
      os[i] = acc;
    }
  }
}

/* ---------------------------------------------------------------------------
 * Transfers: coarse node I (0-based) sits on fine node 2I+1; d-linear
 * interpolation weights 1 (coincident) and 1/2 per axis for neighbours.
 * ------------------------------------------------------------------------- */
static inline double pweight(int dx, int dy, int dz) {
  return (dx ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * (dz ? 0.5 : 1.0);
}

void orc_prolong(const og_grid* g, int nrhs, const ozc* ec, ozc* uf) {
  og_grid c;
  og_coarsen(g, &c);
  const int64_t Nf = og_npts(g), Nc = og_npts(&c);
  memset(uf, 0, sizeof(ozc) * Nf * nrhs);
  for (int s = 0; s < nrhs; ++s) {
    /* Scatter form u_f += P e_c, one coarse node at a time (serial: simple). */
    for (int64_t ci = 0; ci < Nc; ++ci) {
      int X, Y, Z;
      gcoord(&c, ci, &X, &Y, &Z);
      for (int dz = ozlo(g); dz <= ozhi(g); ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            int fx = 2 * X + 1 + dx, fy = 2 * Y + 1 + dy;
            int fz = g->dim == 3 ? 2 * Z + 1 + dz : 0;
            uf[(int64_t)s * Nf + gidx(g, fx, fy, fz)] += pweight(dx, dy, dz) * ec[(int64_t)s * Nc + ci];
          }
    }
  }
}

void orc_restrict(const og_grid* g, int nrhs, const ozc* rf, ozc* rc) {
  og_grid c;
  og_coarsen(g, &c);
  const int64_t Nf = og_npts(g), Nc = og_npts(&c);
  const double scale = 1.0 / (double)(1 << g->dim);
  for (int s = 0; s < nrhs; ++s) {
#pragma omp parallel for schedule(static) if (Nc > 8192)
    for (int64_t ci = 0; ci < Nc; ++ci) {
      int X, Y, Z;
      gcoord(&c, ci, &X, &Y, &Z);
      ozc acc = 0;
      for (int dz = ozlo(g); dz <= ozhi(g); ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            int fx = 2 * X + 1 + dx, fy = 2 * Y + 1 + dy;
            int fz = g->dim == 3 ? 2 * Z + 1 + dz : 0;
            acc += pweight(dx, dy, dz) * rf[(int64_t)s * Nf + gidx(g, fx, fy, fz)];
          }
      rc[(int64_t)s * Nc + ci] = scale * acc;
    }
  }
}

/* ---------------------------------------------------------------------------
 * Galerkin operator R S P, read off by probing. Coarse nodes of one colour
 * (I_a mod 3 fixed) are 3 apart, so R S P applied to their sum gives, at a
 * coarse node J, the single coupling of J to the colour-c node next to it.
 * ------------------------------------------------------------------------- */
void orc_galerkin(const og_grid* g, const ozc* stf, const double* m, const double* gamma,
                  double omega, double beta, ozc* stc) {
  og_grid c;
  og_coarsen(g, &c);
  const int64_t Nf = og_npts(g), Nc = og_npts(&c);
  ozc* e = (ozc*)malloc(sizeof(ozc) * Nc);
  ozc* y = (ozc*)malloc(sizeof(ozc) * Nc);
  ozc* pf = (ozc*)malloc(sizeof(ozc) * Nf);
  ozc* af = (ozc*)malloc(sizeof(ozc) * Nf);
  memset(stc, 0, sizeof(ozc) * Nc * 27);
  for (int cz = 0; cz < (g->dim == 3 ? 3 : 1); ++cz)
    for (int cy = 0; cy < 3; ++cy)
      for (int cx = 0; cx < 3; ++cx) {
        for (int64_t ci = 0; ci < Nc; ++ci) {
          int X, Y, Z;
          gcoord(&c, ci, &X, &Y, &Z);
          int on = (X % 3 == cx) && (Y % 3 == cy) && (g->dim == 2 || Z % 3 == cz);
          e[ci] = on ? 1.0 : 0.0;
        }
        orc_prolong(g, 1, e, pf);
        if (stf)
          orc_apply_stencil(g, stf, 1, pf, af);
        else
          orc_apply_fine(g, m, gamma, omega, beta, 1, pf, af);
        orc_restrict(g, 1, af, y);
        for (int64_t cj = 0; cj < Nc; ++cj) {
          int X, Y, Z;
          gcoord(&c, cj, &X, &Y, &Z);
          for (int oz = ozlo(&c); oz <= ozhi(&c); ++oz)
            for (int oy = -1; oy <= 1; ++oy)
              for (int ox = -1; ox <= 1; ++ox) {
                int ix = X + ox, iy = Y + oy, iz = Z + oz;
                if (!inside(&c, ix, iy, iz)) continue;
                int col = (ix % 3 == cx) && (iy % 3 == cy) && (g->dim == 2 || iz % 3 == cz);
                if (col) stc[cj * 27 + sidx(ox, oy, oz)] = y[cj];
              }
        }
      }
  free(e);
  free(y);
  free(pf);
  free(af);
}

/* ---------------------------------------------------------------------------
 * Damped Jacobi (section 5.3: weight 0.8).
 * ------------------------------------------------------------------------- */
void orc_jacobi(const og_grid* g, const ozc* st, double w, int nsweep, int nrhs,
                const ozc* f, ozc* u) {
  const int64_t N = og_npts(g);
  ozc* r = (ozc*)malloc(sizeof(ozc) * N * nrhs);
  for (int k = 0; k < nsweep; ++k) {
    orc_apply_stencil(g, st, nrhs, u, r);
    for (int s = 0; s < nrhs; ++s)
#pragma omp parallel for schedule(static) if (N > 32768)
      for (int64_t i = 0; i < N; ++i) {
        int64_t j = (int64_t)s * N + i;
        u[j] += w * (f[j] - r[j]) / st[i * 27 + sidx(0, 0, 0)];
      }
  }
  free(r);
}

/* ---------------------------------------------------------------------------
 * Banded LU with partial pivoting (coarsest-grid LU solve). Row i stores the
 * logical columns i-kl .. i-kl+ld-1, ld = 2kl+ku+1 (room for pivot fill).
 * ------------------------------------------------------------------------- */
#define BAND(b, i, j) ((b)->a[(i) * (b)->ld + ((j) - (i) + (b)->kl)])

int orc_band_factor(const og_grid* g, const ozc* st, orc_band* b) {
  const int64_t n = og_npts(g);
  int64_t bw = 1;
  if (g->dim >= 2) bw = (int64_t)g->nu[0] + 1;
  if (g->dim == 3) bw = (int64_t)g->nu[0] * g->nu[1] + g->nu[0] + 1;
  if (bw > n - 1) bw = n - 1 > 0 ? n - 1 : 0;
  b->n = n;
  b->kl = bw;
  b->ku = bw;
  b->ld = 2 * bw + bw + 1;
  b->a = (ozc*)calloc((size_t)(n * b->ld), sizeof(ozc));
  b->piv = (int64_t*)malloc(sizeof(int64_t) * n);
  if (!b->a || !b->piv) return -1;
  for (int64_t i = 0; i < n; ++i) {
    int x, y, z;
    gcoord(g, i, &x, &y, &z);
    for (int oz = ozlo(g); oz <= ozhi(g); ++oz)
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox)
          if (inside(g, x + ox, y + oy, z + oz))
            BAND(b, i, gidx(g, x + ox, y + oy, z + oz)) = st[i * 27 + sidx(ox, oy, oz)];
  }
  /* Row i only ever holds columns < i - kl + ld; the largest column a row can
   * acquire after swaps is k + kl + ku, which fits. */
  for (int64_t k = 0; k < n; ++k) {
    int64_t last = k + b->kl < n - 1 ? k + b->kl : n - 1;
    int64_t p = k;
    double best = cabs(BAND(b, k, k));
    for (int64_t i = k + 1; i <= last; ++i)
      if (cabs(BAND(b, i, k)) > best) {
        best = cabs(BAND(b, i, k));
        p = i;
      }
    b->piv[k] = p;
    if (best == 0.0) return 1;
    int64_t cend = k + b->kl + b->ku < n - 1 ? k + b->kl + b->ku : n - 1;
    if (p != k)
      for (int64_t j = k; j <= cend; ++j) {
        ozc t = BAND(b, k, j);
        BAND(b, k, j) = BAND(b, p, j);
        BAND(b, p, j) = t;
      }
    ozc piv = BAND(b, k, k);
#pragma omp parallel for schedule(static) if ((last - k) * (cend - k) > 65536)
    for (int64_t i = k + 1; i <= last; ++i) {
      ozc l = BAND(b, i, k) / piv;
      BAND(b, i, k) = l;
      if (l != 0)
        for (int64_t j = k + 1; j <= cend; ++j) BAND(b, i, j) -= l * BAND(b, k, j);
    }
  }
  return 0;
}

void orc_band_solve(const orc_band* b, int nrhs, ozc* x) {
  const int64_t n = b->n;
#pragma omp parallel for schedule(dynamic) if (nrhs > 1 && n > 4096)
  for (int s = 0; s < nrhs; ++s) {
    ozc* v = x + (int64_t)s * n;
    for (int64_t k = 0; k < n; ++k) { /* forward: apply P then L */
      int64_t p = b->piv[k];
      if (p != k) {
        ozc t = v[k];
        v[k] = v[p];
        v[p] = t;
      }
      int64_t last = k + b->kl < n - 1 ? k + b->kl : n - 1;
      for (int64_t i = k + 1; i <= last; ++i) v[i] -= BAND(b, i, k) * v[k];
    }
    for (int64_t k = n - 1; k >= 0; --k) { /* backward: U */
      int64_t cend = k + b->kl + b->ku < n - 1 ? k + b->kl + b->ku : n - 1;
      ozc acc = v[k];
      for (int64_t j = k + 1; j <= cend; ++j) acc -= BAND(b, k, j) * v[j];
      v[k] = acc / BAND(b, k, k);
    }
  }
}

void orc_band_free(orc_band* b) {
  free(b->a);
  free(b->piv);
  b->a = NULL;
  b->piv = NULL;
}

/* ---------------------------------------------------------------------------
 * Hierarchy and V-cycle (Algorithm "Two-grid cycle", applied recursively;
 * the W-cycle applies it twice to each coarse problem but the coarsest).
 * Level 0 is the shifted fine operator, defined directly from (m, gamma);
 * levels >= 1 are Galerkin stencils; the last level is solved by LU.
 * ------------------------------------------------------------------------- */
struct orc_hier {
  int levels;
  int coarse_kind, coarse_iters;
  int coarse_restarts; /* GMRES cycles of coarse_iters steps (restarted GMRES); 0 or 1: one */
  int cycle_w;         /* 1: W-cycle (two coarse cycles where the coarse level is not the coarsest) */
  int cycle_k;         /* 1: K-cycle (two flexible GMRES steps on such a coarse level) */
  og_grid g[8];
  ozc* st[8];   /* st[0] = shifted fine operator as a stencil */
  int nu_pre[8], nu_post[8];
  double w[8];
  orc_band lu;
  const double *m, *gamma;
  double omega, beta;
  double* mcopy;
  double* gcopy;
};

orc_hier* orc_setup(const og_grid* g, const double* m, const double* gamma, double omega,
                    double beta, int levels, const int* nu_pre, const int* nu_post,
                    const double* wjac, int coarse_kind, int coarse_iters) {
  if (levels < 1 || levels > 8) return NULL;
  orc_hier* H = (orc_hier*)calloc(1, sizeof(orc_hier));
  const int64_t N = og_npts(g);
  H->levels = levels;
  H->coarse_kind = coarse_kind;
  H->coarse_iters = coarse_iters;
  H->omega = omega;
  H->beta = beta;
  H->mcopy = (double*)malloc(sizeof(double) * N);
  H->gcopy = (double*)malloc(sizeof(double) * N);
  memcpy(H->mcopy, m, sizeof(double) * N);
  memcpy(H->gcopy, gamma, sizeof(double) * N);
  H->m = H->mcopy;
  H->gamma = H->gcopy;
  H->g[0] = *g;
  for (int l = 0; l < levels; ++l) {
    H->nu_pre[l] = nu_pre ? nu_pre[l] : 2;
    H->nu_post[l] = nu_post ? nu_post[l] : 2;
    H->w[l] = wjac ? wjac[l] : 0.8;
  }
  H->st[0] = (ozc*)malloc(sizeof(ozc) * N * 27);
  orc_fine_stencil(g, m, gamma, omega, beta, H->st[0]);
  for (int l = 1; l < levels; ++l) {
    og_coarsen(&H->g[l - 1], &H->g[l]);
    H->st[l] = (ozc*)malloc(sizeof(ozc) * og_npts(&H->g[l]) * 27);
    if (l == 1)
      orc_galerkin(&H->g[0], NULL, H->m, H->gamma, omega, beta, H->st[1]);
    else
      orc_galerkin(&H->g[l - 1], H->st[l - 1], NULL, NULL, 0, 0, H->st[l]);
  }
  if (coarse_kind == ORC_COARSE_LU && orc_band_factor(&H->g[levels - 1], H->st[levels - 1], &H->lu) != 0) {
    orc_free(H);
    return NULL;
  }
  return H;
}

void orc_free(orc_hier* H) {
  if (!H) return;
  for (int l = 0; l < H->levels; ++l) free(H->st[l]);
  orc_band_free(&H->lu);
  free(H->mcopy);
  free(H->gcopy);
  free(H);
}

int orc_levels(const orc_hier* H) { return H->levels; }
void orc_level_grid(const orc_hier* H, int l, og_grid* g) { *g = H->g[l]; }
void orc_level_stencil(const orc_hier* H, int l, ozc* st) {
  memcpy(st, H->st[l], sizeof(ozc) * og_npts(&H->g[l]) * 27);
}

static double vnorm(int64_t n, const ozc* x);

/* k steps of GMRES (Arnoldi with modified Gram-Schmidt, least squares by
 * Householder) on the coarsest stencil operator, from u = 0, per column. */
static void coarse_gmres(const og_grid* g, const ozc* st, int k, const ozc* f, ozc* u) {
  const int64_t n = og_npts(g);
  memset(u, 0, sizeof(ozc) * n);
  double beta = vnorm(n, f);
  if (beta == 0.0 || k < 1) return;
  ozc* V = (ozc*)malloc(sizeof(ozc) * n * (k + 1));
  ozc* Hm = (ozc*)calloc((size_t)(k + 1) * k, sizeof(ozc)); /* column-major (k+1) x k */
  for (int64_t i = 0; i < n; ++i) V[i] = f[i] / beta;
  int j;
  for (j = 0; j < k; ++j) {
    ozc* w = V + (int64_t)(j + 1) * n;
    orc_apply_stencil(g, st, 1, V + (int64_t)j * n, w);
    for (int i = 0; i <= j; ++i) {
      ozc d = 0;
      const ozc* vi = V + (int64_t)i * n;
      for (int64_t t = 0; t < n; ++t) d += conj(vi[t]) * w[t];
      Hm[(int64_t)j * (k + 1) + i] = d;
      for (int64_t t = 0; t < n; ++t) w[t] -= d * vi[t];
    }
    double hn = vnorm(n, w);
    Hm[(int64_t)j * (k + 1) + j + 1] = hn;
    if (hn == 0.0) {
      ++j;
      break;
    }
    for (int64_t t = 0; t < n; ++t) w[t] /= hn;
  }
  const int steps = j;
  /* least squares on the leading (steps+1) x steps block */
  ozc* A = (ozc*)malloc(sizeof(ozc) * (steps + 1) * steps);
  ozc* B = (ozc*)calloc((size_t)(steps + 1), sizeof(ozc));
  ozc* y = (ozc*)malloc(sizeof(ozc) * steps);
  double res;
  for (int c = 0; c < steps; ++c)
    for (int r = 0; r <= steps; ++r) A[(int64_t)c * (steps + 1) + r] = Hm[(int64_t)c * (k + 1) + r];
  B[0] = beta;
  orc_lstsq(steps + 1, steps, 1, A, B, y, &res);
  for (int c = 0; c < steps; ++c)
    for (int64_t t = 0; t < n; ++t) u[t] += V[(int64_t)c * n + t] * y[c];
  free(A);
  free(B);
  free(y);
  free(V);
  free(Hm);
}

void orc_set_coarse_restarts(orc_hier* H, int restarts) { H->coarse_restarts = restarts; }
void orc_set_cycle_w(orc_hier* H, int w) { H->cycle_w = w; }
void orc_set_cycle_k(orc_hier* H, int k) { H->cycle_k = k; }

void orc_coarse_solve(const orc_hier* H, int nrhs, const ozc* f, ozc* u) {
  const int l = H->levels - 1;
  const int64_t n = og_npts(&H->g[l]);
  if (H->coarse_kind == ORC_COARSE_LU) {
    memcpy(u, f, sizeof(ozc) * n * nrhs);
    orc_band_solve(&H->lu, nrhs, u);
  } else if (H->coarse_kind == ORC_COARSE_GMRES) {
    /* restarted GMRES(k): the first cycle from zero, each further one on the
     * current residual, its correction added (section 5.3, GMRES-based
     * coarsest solver) */
#pragma omp parallel for schedule(dynamic) if (nrhs > 1 && n > 4096)
    for (int s = 0; s < nrhs; ++s) {
      const ozc* fs = f + (int64_t)s * n;
      ozc* us = u + (int64_t)s * n;
      coarse_gmres(&H->g[l], H->st[l], H->coarse_iters, fs, us);
      if (H->coarse_restarts > 1) {
        ozc* r = (ozc*)malloc(sizeof(ozc) * n);
        ozc* d = (ozc*)malloc(sizeof(ozc) * n);
        for (int q = 1; q < H->coarse_restarts; ++q) {
          orc_apply_stencil(&H->g[l], H->st[l], 1, us, r);
          for (int64_t t = 0; t < n; ++t) r[t] = fs[t] - r[t];
          coarse_gmres(&H->g[l], H->st[l], H->coarse_iters, r, d);
          for (int64_t t = 0; t < n; ++t) us[t] += d[t];
        }
        free(r);
        free(d);
      }
    }
  } else {
    /* relaxation only: nu_pre + nu_post damped Jacobi sweeps from zero */
    int sweeps = H->nu_pre[l] + H->nu_post[l];
    if (sweeps < 1) sweeps = 1;
    memset(u, 0, sizeof(ozc) * n * nrhs);
    orc_jacobi(&H->g[l], H->st[l], H->w[l], sweeps, nrhs, f, u);
  }
}

/* Level-0 operator apply uses the definition from (m, gamma); coarser
 * levels use their Galerkin stencils. */
static void level_apply(const orc_hier* H, int l, int nrhs, const ozc* u, ozc* out) {
  if (l == 0)
    orc_apply_fine(&H->g[0], H->m, H->gamma, H->omega, H->beta, nrhs, u, out);
  else
    orc_apply_stencil(&H->g[l], H->st[l], nrhs, u, out);
}

static void level_jacobi(const orc_hier* H, int l, int nsweep, int nrhs, const ozc* f, ozc* u) {
  const og_grid* g = &H->g[l];
  const int64_t N = og_npts(g);
  ozc* r = (ozc*)malloc(sizeof(ozc) * N * nrhs);
  for (int k = 0; k < nsweep; ++k) {
    level_apply(H, l, nrhs, u, r);
    for (int s = 0; s < nrhs; ++s)
#pragma omp parallel for schedule(static) if (N > 32768)
      for (int64_t i = 0; i < N; ++i) {
        int64_t j = (int64_t)s * N + i;
        u[j] += H->w[l] * (f[j] - r[j]) / H->st[l][i * 27 + sidx(0, 0, 0)];
      }
  }
  free(r);
}

static void vcycle_rec(const orc_hier* H, int l, int nrhs, const ozc* f, ozc* u);

/* K-cycle coarse correction (Notay and Vassilevski's recursive Krylov
 * cycle; the paper's K-FGMRES, section 5.3): the coarse problem M_l e = f is
 * solved by two iterations of flexible GMRES from e = 0, each step
 * preconditioned by the cycle of level l, one column at a time:
 *   v1 = f / ||f||, z1 = B v1, w = M z1, h11 = v1^H w, w -= h11 v1,
 *   h21 = ||w||, v2 = w / h21, z2 = B v2, w = M z2, h12 = v1^H w,
 *   w -= h12 v1, h22 = v2^H w, w -= h22 v2, h32 = ||w||,
 *   y = argmin || ||f|| e1 - H y ||, e = z1 y1 + z2 y2
 * (a vanishing h21 ends after one step). */
static void kcycle_coarse(const orc_hier* H, int l, int nrhs, const ozc* f, ozc* e) {
  const int64_t n = og_npts(&H->g[l]);
  ozc* v = (ozc*)malloc(sizeof(ozc) * n * 2);
  ozc* z = (ozc*)malloc(sizeof(ozc) * n * 2);
  ozc* w = (ozc*)malloc(sizeof(ozc) * n);
  for (int s = 0; s < nrhs; ++s) {
    const ozc* fs = f + (int64_t)s * n;
    ozc* es = e + (int64_t)s * n;
    memset(es, 0, sizeof(ozc) * n);
    const double beta = vnorm(n, fs);
    if (beta == 0.0) continue;
    ozc Hm[6] = {0, 0, 0, 0, 0, 0}; /* column-major 3 x 2 */
    for (int64_t i = 0; i < n; ++i) v[i] = fs[i] / beta;
    int steps = 2;
    for (int j = 0; j < 2; ++j) {
      vcycle_rec(H, l, 1, v + (int64_t)j * n, z + (int64_t)j * n);
      orc_apply_stencil(&H->g[l], H->st[l], 1, z + (int64_t)j * n, w);
      for (int i = 0; i <= j; ++i) {
        const ozc* vi = v + (int64_t)i * n;
        ozc d = 0;
        for (int64_t t = 0; t < n; ++t) d += conj(vi[t]) * w[t];
        Hm[j * 3 + i] = d;
        for (int64_t t = 0; t < n; ++t) w[t] -= d * vi[t];
      }
      const double hn = vnorm(n, w);
      Hm[j * 3 + j + 1] = hn;
      if (j == 0) {
        if (hn == 0.0) {
          steps = 1;
          break;
        }
        for (int64_t t = 0; t < n; ++t) v[n + t] = w[t] / hn;
      }
    }
    ozc A[6], B[3] = {beta, 0, 0}, y[2];
    double res;
    for (int c = 0; c < steps; ++c)
      for (int r = 0; r <= steps; ++r) A[c * (steps + 1) + r] = Hm[c * 3 + r];
    orc_lstsq(steps + 1, steps, 1, A, B, y, &res);
    for (int c = 0; c < steps; ++c)
      for (int64_t t = 0; t < n; ++t) es[t] += z[(int64_t)c * n + t] * y[c];
  }
  free(v);
  free(z);
  free(w);
}

static void vcycle_rec(const orc_hier* H, int l, int nrhs, const ozc* f, ozc* u) {
  const int64_t N = og_npts(&H->g[l]);
  if (l == H->levels - 1) {
    orc_coarse_solve(H, nrhs, f, u);
    return;
  }
  const int64_t Nc = og_npts(&H->g[l + 1]);
  memset(u, 0, sizeof(ozc) * N * nrhs);
  level_jacobi(H, l, H->nu_pre[l], nrhs, f, u);           /* 1. pre-relax */
  ozc* r = (ozc*)malloc(sizeof(ozc) * N * nrhs);
  level_apply(H, l, nrhs, u, r);                           /* 2. r = f - A u */
  for (int64_t j = 0; j < N * nrhs; ++j) r[j] = f[j] - r[j];
  ozc* rc = (ozc*)malloc(sizeof(ozc) * Nc * nrhs);
  ozc* ec = (ozc*)malloc(sizeof(ozc) * Nc * nrhs);
  orc_restrict(&H->g[l], nrhs, r, rc);                     /*    r_c = R r */
  if (H->cycle_k && l + 1 < H->levels - 1)
    kcycle_coarse(H, l + 1, nrhs, rc, ec);                 /* 3. coarse problem: K-cycle */
  else
    vcycle_rec(H, l + 1, nrhs, rc, ec);                    /* 3. coarse problem */
  if (H->cycle_w && l + 1 < H->levels - 1) {
    /* W-cycle: the coarse problem gets a second cycle, on the residual the
     * first one left: e_c += B_c (r_c - M_c e_c). The coarsest level is
     * solved once. */
    const int64_t n2 = Nc * nrhs;
    ozc* r2 = (ozc*)malloc(sizeof(ozc) * n2);
    ozc* d2 = (ozc*)malloc(sizeof(ozc) * n2);
    level_apply(H, l + 1, nrhs, ec, r2);
    for (int64_t j = 0; j < n2; ++j) r2[j] = rc[j] - r2[j];
    vcycle_rec(H, l + 1, nrhs, r2, d2);
    for (int64_t j = 0; j < n2; ++j) ec[j] += d2[j];
    free(r2);
    free(d2);
  }
  orc_prolong(&H->g[l], nrhs, ec, r);                      /* 4. u += P e_c */
  for (int64_t j = 0; j < N * nrhs; ++j) u[j] += r[j];
  level_jacobi(H, l, H->nu_post[l], nrhs, f, u);          /* 5. post-relax */
  free(r);
  free(rc);
  free(ec);
}

void orc_vcycle(const orc_hier* H, int nrhs, const ozc* f, ozc* u) {
  vcycle_rec(H, 0, nrhs, f, u);
}

/* ---------------------------------------------------------------------------
 * Dense helpers: complex Householder QR and least squares.
 * ------------------------------------------------------------------------- */
static double vnorm(int64_t n, const ozc* x) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += creal(x[i]) * creal(x[i]) + cimag(x[i]) * cimag(x[i]);
  return sqrt(s);
}

/* Reflector I - 2 v v^H that maps x to alpha e1, |alpha| = ||x||. Returns
 * 0 if x is zero (no reflection). */
static int make_reflector(int64_t n, const ozc* x, ozc* v, ozc* alpha) {
  double nx = vnorm(n, x);
  if (nx == 0.0) {
    *alpha = 0;
    return 0;
  }
  ozc ph = cabs(x[0]) > 0 ? x[0] / cabs(x[0]) : 1.0;
  *alpha = -ph * nx;
  memcpy(v, x, sizeof(ozc) * n);
  v[0] -= *alpha;
  double nv = vnorm(n, v);
  for (int64_t i = 0; i < n; ++i) v[i] /= nv;
  return 1;
}

/* y <- (I - 2 v v^H) y on a vector of length n. */
static void apply_reflector(int64_t n, const ozc* v, ozc* y) {
  ozc d = 0;
  for (int64_t i = 0; i < n; ++i) d += conj(v[i]) * y[i];
  for (int64_t i = 0; i < n; ++i) y[i] -= 2.0 * v[i] * d;
}

void orc_householder_qr(int64_t N, int p, ozc* A, ozc* R) {
  ozc* V = (ozc*)calloc((size_t)(N * p), sizeof(ozc));
  int* has = (int*)calloc(p, sizeof(int));
  for (int k = 0; k < p; ++k) {
    ozc alpha;
    ozc* vk = V + (int64_t)k * N;
    has[k] = make_reflector(N - k, A + (int64_t)k * N + k, vk, &alpha);
    if (has[k]) {
#pragma omp parallel for schedule(static) if (N > 32768 && p > 1)
      for (int j = k; j < p; ++j) apply_reflector(N - k, vk, A + (int64_t)j * N + k);
    }
  }
  for (int j = 0; j < p; ++j)
    for (int i = 0; i < p; ++i) R[(int64_t)j * p + i] = i <= j ? A[(int64_t)j * N + i] : 0;
  /* Q = H_0 ... H_{p-1} [I; 0] */
  for (int j = 0; j < p; ++j) {
    ozc* q = A + (int64_t)j * N;
    memset(q, 0, sizeof(ozc) * N);
    q[j] = 1.0;
  }
  for (int k = p - 1; k >= 0; --k)
    if (has[k]) {
#pragma omp parallel for schedule(static) if (N > 32768 && p > 1)
      for (int j = 0; j < p; ++j) apply_reflector(N - k, V + (int64_t)k * N, A + (int64_t)j * N + k);
    }
  free(V);
  free(has);
}

/* Rank-revealing Householder QR with column pivoting: at step k the
 * remaining column of largest norm (rows k..N-1) is brought to position k;
 * the factorisation stops when that norm is at most tol times the largest
 * initial column norm (rank r = k). A (N x p, column-major) is replaced by
 * Q with orthonormal columns 0..r-1 and zero columns r..p-1; R (p x p,
 * column-major) gets rows 0..r-1 of the pivoted factor with its columns
 * put back in the original order and zero rows r..p-1, so that the input
 * equals Q R to within tol. Returns r. A block whose columns are
 * dependent (duplicate sources) thus keeps only independent directions. */
int orc_householder_qr_rr(int64_t N, int p, ozc* A, ozc* R, double tol) {
  ozc* V = (ozc*)calloc((size_t)(N * p), sizeof(ozc));
  int* perm = (int*)malloc(sizeof(int) * p);
  double nmax = 0.0;
  for (int j = 0; j < p; ++j) {
    perm[j] = j;
    nmax = fmax(nmax, vnorm(N, A + (int64_t)j * N));
  }
  int r = 0;
  for (int k = 0; k < p && k < N; ++k) {
    int jm = k;
    double best = -1.0;
    for (int j = k; j < p; ++j) {
      const double nj = vnorm(N - k, A + (int64_t)j * N + k);
      if (nj > best) {
        best = nj;
        jm = j;
      }
    }
    if (!(best > tol * nmax)) break;
    if (jm != k) {
      for (int64_t i = 0; i < N; ++i) {
        const ozc t = A[(int64_t)k * N + i];
        A[(int64_t)k * N + i] = A[(int64_t)jm * N + i];
        A[(int64_t)jm * N + i] = t;
      }
      const int t = perm[k];
      perm[k] = perm[jm];
      perm[jm] = t;
    }
    ozc alpha;
    make_reflector(N - k, A + (int64_t)k * N + k, V + (int64_t)k * N, &alpha);
    for (int j = k; j < p; ++j) apply_reflector(N - k, V + (int64_t)k * N, A + (int64_t)j * N + k);
    r = k + 1;
  }
  for (int j = 0; j < p; ++j)
    for (int i = 0; i < p; ++i) R[(int64_t)perm[j] * p + i] = (i < r && i <= j) ? A[(int64_t)j * N + i] : 0;
  /* Q = H_0 ... H_{r-1} [I_r; 0], zero columns beyond the rank */
  for (int j = 0; j < p; ++j) {
    ozc* q = A + (int64_t)j * N;
    memset(q, 0, sizeof(ozc) * N);
    if (j < r) q[j] = 1.0;
  }
  for (int k = r - 1; k >= 0; --k)
    for (int j = 0; j < r; ++j) apply_reflector(N - k, V + (int64_t)k * N, A + (int64_t)j * N + k);
  free(V);
  free(perm);
  return r;
}

void orc_lstsq(int mr, int nc, int k, const ozc* A, const ozc* B, ozc* Y, double* res) {
  ozc* a = (ozc*)malloc(sizeof(ozc) * mr * nc);
  ozc* b = (ozc*)malloc(sizeof(ozc) * mr * k);
  ozc* v = (ozc*)malloc(sizeof(ozc) * mr);
  memcpy(a, A, sizeof(ozc) * mr * nc);
  memcpy(b, B, sizeof(ozc) * mr * k);
  for (int j = 0; j < nc; ++j) { /* QR of A, applied to B on the fly */
    ozc alpha;
    if (!make_reflector(mr - j, a + (int64_t)j * mr + j, v, &alpha)) continue;
    for (int c = j; c < nc; ++c) apply_reflector(mr - j, v, a + (int64_t)c * mr + j);
    for (int c = 0; c < k; ++c) apply_reflector(mr - j, v, b + (int64_t)c * mr + j);
  }
  for (int c = 0; c < k; ++c) { /* back substitution with R = a[0:nc, 0:nc] */
    for (int i = nc - 1; i >= 0; --i) {
      ozc acc = b[(int64_t)c * mr + i];
      for (int j = i + 1; j < nc; ++j) acc -= a[(int64_t)j * mr + i] * Y[(int64_t)c * nc + j];
      /* a column of zeros (a direction dropped by the rank-revealing QR)
       * does not change the residual: its coefficient is taken as 0 */
      Y[(int64_t)c * nc + i] = a[(int64_t)i * mr + i] != 0 ? acc / a[(int64_t)i * mr + i] : 0;
    }
    res[c] = vnorm(mr - nc, b + (int64_t)c * mr + nc);
  }
  free(a);
  free(b);
  free(v);
}

/* ---------------------------------------------------------------------------
 * Block FGMRES(m) (section 5.3), right-preconditioned by the V-cycle.
 * ------------------------------------------------------------------------- */
int orc_block_fgmres(const orc_hier* Hh, int use_prec, int p, const ozc* Q, ozc* X, int warm,
                     double tol, int restart, int maxit, int* iters, double* relres,
                     double* hist) {
  const int64_t N = og_npts(&Hh->g[0]);
  const int mm = restart;
  const int64_t blk = N * p;
  ozc* V = (ozc*)malloc(sizeof(ozc) * blk * (mm + 1));
  ozc* Z = (ozc*)malloc(sizeof(ozc) * blk * mm);
  ozc* W = (ozc*)malloc(sizeof(ozc) * blk);
  const int hr = (mm + 1) * p, hc = mm * p;
  ozc* Hb = (ozc*)calloc((size_t)hr * hc, sizeof(ozc)); /* column-major (mm+1)p x mm p */
  ozc* S = (ozc*)malloc(sizeof(ozc) * p * p);
  ozc* Hij = (ozc*)malloc(sizeof(ozc) * p * p);
  double* qn = (double*)malloc(sizeof(double) * p);
  double* est = (double*)malloc(sizeof(double) * p);
  int it = 0, done = 0;
  for (int s = 0; s < p; ++s) qn[s] = vnorm(N, Q + (int64_t)s * N);
  if (!warm) memset(X, 0, sizeof(ozc) * blk);
  while (!done) {
    /* R = Q - H X, checked column-wise in FP64 */
    orc_apply_fine(&Hh->g[0], Hh->m, Hh->gamma, Hh->omega, 0.0, p, X, V);
    int all = 1;
    for (int s = 0; s < p; ++s) {
      for (int64_t i = 0; i < N; ++i) V[(int64_t)s * N + i] = Q[(int64_t)s * N + i] - V[(int64_t)s * N + i];
      relres[s] = qn[s] > 0 ? vnorm(N, V + (int64_t)s * N) / qn[s] : 0.0;
      if (relres[s] > tol) all = 0;
    }
    if (all || it >= maxit) {
      done = 1;
      break;
    }
    /* R = V_1 S; dependent residual columns (e.g. duplicate sources) keep
     * only their independent directions (zero columns of V_1) */
    orc_householder_qr_rr(N, p, V, S, 1e-13);
    memset(Hb, 0, sizeof(ozc) * hr * hc);
    int j;
    for (j = 0; j < mm && it < maxit; ++j) {
      ozc* Vj = V + (int64_t)j * blk;
      ozc* Zj = Z + (int64_t)j * blk;
      if (use_prec)
        orc_vcycle(Hh, p, Vj, Zj);
      else
        memcpy(Zj, Vj, sizeof(ozc) * blk);
      orc_apply_fine(&Hh->g[0], Hh->m, Hh->gamma, Hh->omega, 0.0, p, Zj, W);
      for (int i = 0; i <= j; ++i) { /* block modified Gram-Schmidt */
        const ozc* Vi = V + (int64_t)i * blk;
        for (int b = 0; b < p; ++b)
          for (int a = 0; a < p; ++a) {
            ozc acc = 0;
            const ozc* va = Vi + (int64_t)a * N;
            const ozc* wb = W + (int64_t)b * N;
#pragma omp parallel for reduction(+ : acc) schedule(static) if (N > 32768)
            for (int64_t n = 0; n < N; ++n) acc += conj(va[n]) * wb[n];
            Hij[b * p + a] = acc;
          }
        for (int b = 0; b < p; ++b) {
          ozc* wb = W + (int64_t)b * N;
#pragma omp parallel for schedule(static) if (N > 32768)
          for (int64_t n = 0; n < N; ++n) {
            ozc acc = 0;
            for (int a = 0; a < p; ++a) acc += Vi[(int64_t)a * N + n] * Hij[b * p + a];
            wb[n] -= acc;
          }
        }
        for (int b = 0; b < p; ++b)
          for (int a = 0; a < p; ++a) Hb[(int64_t)(j * p + b) * hr + i * p + a] = Hij[b * p + a];
      }
      ozc* Vn = V + (int64_t)(j + 1) * blk;
      memcpy(Vn, W, sizeof(ozc) * blk);
      orc_householder_qr_rr(N, p, Vn, Hij, 1e-13); /* W = V_{j+1} H_{j+1,j} */
      for (int b = 0; b < p; ++b)
        for (int a = 0; a < p; ++a) Hb[(int64_t)(j * p + b) * hr + (j + 1) * p + a] = Hij[b * p + a];
      it++;
      /* least squares on the leading (j+2)p x (j+1)p block, residual estimates */
      int r = (j + 2) * p, c = (j + 1) * p;
      ozc* A = (ozc*)malloc(sizeof(ozc) * r * c);
      ozc* B = (ozc*)calloc((size_t)r * p, sizeof(ozc));
      ozc* Y = (ozc*)malloc(sizeof(ozc) * c * p);
      for (int cc = 0; cc < c; ++cc)
        for (int rr = 0; rr < r; ++rr) A[(int64_t)cc * r + rr] = Hb[(int64_t)cc * hr + rr];
      for (int b = 0; b < p; ++b)
        for (int a = 0; a < p; ++a) B[(int64_t)b * r + a] = S[b * p + a];
      orc_lstsq(r, c, p, A, B, Y, est);
      double worst = 0.0;
      int conv = 1;
      for (int s = 0; s < p; ++s) {
        double e = qn[s] > 0 ? est[s] / qn[s] : 0.0;
        if (e > worst) worst = e;
        if (e > tol) conv = 0;
      }
      if (hist) hist[it - 1] = worst;
      if (conv || j == mm - 1 || it >= maxit) { /* X += [Z_1..Z_{j+1}] Y */
        for (int s = 0; s < p; ++s) {
          ozc* xs = X + (int64_t)s * N;
#pragma omp parallel for schedule(static) if (N > 32768)
          for (int64_t n = 0; n < N; ++n) {
            ozc acc = 0;
            for (int cc = 0; cc < c; ++cc) {
              int jj = cc / p, a = cc % p;
              acc += Z[(int64_t)jj * blk + (int64_t)a * N + n] * Y[(int64_t)s * c + cc];
            }
            xs[n] += acc;
          }
        }
        free(A);
        free(B);
        free(Y);
        break;
      }
      free(A);
      free(B);
      free(Y);
    }
  }
  *iters = it;
  int ok = 1;
  for (int s = 0; s < p; ++s)
    if (relres[s] > tol) ok = 0;
  free(V);
  free(Z);
  free(W);
  free(Hb);
  free(S);
  free(Hij);
  free(qn);
  free(est);
  return ok ? 0 : 1;
}
