// helm.cpp -- host side of the solver: the C ABI of include/helm.h, the
// multigrid hierarchy, the cycle scheduler and the block FGMRES driver.
// Every arithmetic step runs in the HIP kernels of k_level / k_setup /
// k_krylov; this file only sequences launches, owns device memory and
// reads back the p per-column residual estimates once per Arnoldi step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <string>
#include <thread>
#include <vector>

#include "../../include/helm.h"
#include "kernels.hpp"
#include "learned.hpp"

namespace helm {

[[noreturn]] void fatal_combo(const char* where) {
  std::fprintf(stderr, "helm: unsupported precision combination in %s\n", where);
  std::abort();
}

hipError_t dmalloc_raw(void** p, size_t bytes) {
  const hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess || bytes == 0) return e;
  const char* v = std::getenv("HELM_SENTINEL");
  if (v && v[0] == '1') {
    // synchronous fill before the memory is handed out
    const hipError_t f = hipMemset(*p, 0xFF, bytes);
    if (f != hipSuccess) return f;
    return hipDeviceSynchronize();
  }
  return hipSuccess;
}

static thread_local std::string g_err;

helm_status fail(helm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HCHECK(expr)                                                                              \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess)                                                                         \
      return fail(e_ == hipErrorOutOfMemory ? HELM_ERR_OOM : HELM_ERR_DEVICE, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                              \
  } while (0)

static size_t psize(Prec p) { return p == P64 ? 16 : (p == P32 ? 8 : 4); }

struct Level {
  int nu[3] = {1, 1, 1};
  double h[3] = {1, 1, 1};
  double ih[3] = {0, 0, 0};  // 1/h^2
  int64_t npts = 0;
  // coefficients: fine level uses diagonals, coarser levels stencils [N][NS]
  c128* dH = nullptr;
  c128* dM = nullptr;
  c128* dS = nullptr;  // finest level: omega^2 (1 - i gamma), the sensitivity factor
  c128* dw64 = nullptr;
  c64* dM32 = nullptr;
  c64* dw32 = nullptr;
  c128* st64 = nullptr;
  c64* st32 = nullptr;
  // per-solve fields [N][P]
  void* F = nullptr;
  void* U0 = nullptr;
  void* U1 = nullptr;
  void* Rr = nullptr;
  Prec pf = P64;  // field storage precision
  Geo geo(int P) const {
    Geo g;
    g.nx = nu[0];
    g.ny = nu[1];
    g.nz = nu[2];
    g.npts = npts;
    g.P = P;
    return g;
  }
};

}  // namespace helm

using namespace helm;

struct helm_net_s;

struct helm_ctx {
  int dim = 3;
  int L = 0;
  int precision = HELM_FP64;
  int coarse = HELM_COARSE_LU;
  int cycle = HELM_CYCLE_V;
  int coarse_iters = 20;
  int coarse_restarts = 1;  // GMRES cycles of coarse_iters steps on the coarsest grid
  // coarsest GMRES storage: basis, Hessenberg, coefficients
  void* cg_mem = nullptr;
  int cg_P = 0;
  int nu_pre[HELM_MAX_LEVELS], nu_post[HELM_MAX_LEVELS];
  double wj[HELM_MAX_LEVELS];
  double omega = 0, shift = 0;
  Level lv[HELM_MAX_LEVELS];
  int64_t nc = 0;          // coarsest unknowns
  c128* Minv64 = nullptr;  // dense coarsest inverse
  c64* Minv32 = nullptr;
  learned::Net* net = nullptr;
  int64_t fallbacks = 0;            // learned coarsest solves replaced by GMRES
  learned::Net* cap = nullptr;      // pool receiving coarsest (f, e) pairs
  helm_net_s* capw = nullptr;       // the network object that owns `cap`
  // cycles captured as HIP graphs, keyed by block width and buffers
  struct CycleGraph {
    int P;
    const void* f;
    void* out;
    void* tmp;
    hipGraphExec_t exec;
  };
  uint64_t graph_net_gen = 0;     // network scratch generation the graphs were taken with
  std::vector<CycleGraph> graphs;
  // persistent cycles: the recorded phases of a cycle per (block width, buffers)
  struct CyclePlan {
    int P;
    const void* f;
    void* out;
    void* tmp;
    Phase* d;  // device copy of the phases
    int nph, grid;
  };
  std::vector<CyclePlan> plans;
  std::vector<Phase>* plan = nullptr;  // set while a cycle is being recorded
  bool plan_bad = false;               // the recorded cycle has a step the persistent kernel lacks
  hipStream_t gstream = nullptr;  // capture stream (never executes work itself)
  hipStream_t bstream = nullptr;  // this handle's stream inside helm_solve_batch
  bool capturing = false;         // a cycle is being recorded into a graph
  bool force_fallback = false;    // redo a cycle with the GMRES coarsest fallback
  bool rate_fallback = false;     // the rate check switched this solve to the fallback
  // cached per-solve field allocation
  int fieldsP = 0;
  void* fieldmem = nullptr;
  // partial sums of helm_residual (allocated on its first call)
  double* resid_buf = nullptr;
  // adjoint solutions of helm_jtvp (allocated on its first call)
  void* sensbuf = nullptr;
  size_t sensbytes = 0;
  // cached Krylov workspace
  void* ws = nullptr;
  size_t wsbytes = 0;
  // per-level field-sized scratch (allocated with the fields): the second
  // coarse cycle's right-hand side of the W-cycle, z2 of the K-cycle
  std::vector<void*> kbuf;
  // K-cycle: per coarse level, three vectors (v1, v2, w) in the cycle's
  // arithmetic precision and the per-column Hessenberg / least-squares data
  void* kmem = nullptr;
  std::vector<char*> klev;
  double* hbuf = nullptr;  // pinned host scratch
  size_t hbufn = 0;
  // tuned tile of the finest-level marching kernel, per block width P
  int tileP = 0;
  FineTile tile = {4, 32};
  // per-class kernel timing
  bool prof = false;
  std::vector<hipEvent_t> evpool;
  std::vector<int> evcls;
  size_t evused = 0;
};

namespace helm {

// Records a HIP event pair around the launches in its scope when timing is on.
struct Prof {
  helm_ctx* c;
  hipStream_t s;
  size_t idx = 0;
  bool on;
  Prof(helm_ctx* c_, int cls, hipStream_t s_) : c(c_), s(s_), on(c_->prof) {
    if (!on) return;
    if (c->evused + 2 > c->evpool.size()) {
      for (int k = 0; k < 256; ++k) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) {
          on = false;
          return;
        }
        c->evpool.push_back(e);
      }
    }
    idx = c->evused;
    c->evused += 2;
    c->evcls.push_back(cls);
    hipEventRecord(c->evpool[idx], s);
  }
  ~Prof() {
    if (on) hipEventRecord(c->evpool[idx + 1], s);
  }
};

static Prec field_prec(const helm_ctx* c, int l) {
  if (c->precision == HELM_FP64) return P64;
  if (l == 0) return P32;
  if (l == c->L - 1) return P32;  // coarsest vectors stay FP32 (dense solve input)
  return PBF;
}
static Prec comp_prec(const helm_ctx* c) { return c->precision == HELM_FP64 ? P64 : P32; }

static const void* level_st(const helm_ctx* c, int l) {
  return c->precision == HELM_FP64 ? (const void*)c->lv[l].st64 : (const void*)c->lv[l].st32;
}
static const void* level_dw(const helm_ctx* c, int l) {
  return c->precision == HELM_FP64 ? (const void*)c->lv[l].dw64 : (const void*)c->lv[l].dw32;
}

__global__ void k_add_c128(int64_t n, const c128* __restrict__ x, c128* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = c128{y[i].re + x[i].re, y[i].im + x[i].im};
}

// One relaxation-family launch on level l (mode as launch_fine).
static void level_op(helm_ctx* c, int l, int mode, int P, const void* u, const void* f, void* out, hipStream_t s) {
  if (c->plan) {
    const Level& L = c->lv[l];
    Phase q{};
    q.op = l == 0 ? PH_FINE : PH_GAL;
    q.mode = mode;
    q.pa = field_prec(c, l);
    q.pb = comp_prec(c);
    q.g = L.geo(P);
    q.u = u;
    q.f = f;
    q.out = out;
    if (l == 0) {
      q.c0 = c->precision == HELM_FP64 ? (const void*)L.dM : (const void*)L.dM32;
      for (int a = 0; a < 3; ++a) q.ih[a] = L.ih[a];
    } else {
      q.c0 = level_st(c, l);
    }
    q.c1 = level_dw(c, l);
    c->plan->push_back(q);
    return;
  }
  Prof pr(c,
          l == 0 ? (mode == 1 ? HELM_K_FINE_RESID : (mode == 3 ? HELM_K_FINE_SWEEP0 : HELM_K_FINE_SWEEP))
                 : HELM_K_COARSE_SWEEP,
          s);
  const Level& L = c->lv[l];
  const Prec pf = field_prec(c, l), pt = comp_prec(c);
  if (l == 0) {
    const void* diag = c->precision == HELM_FP64 ? (const void*)L.dM : (const void*)L.dM32;
    launch_fine(mode, pf, pf, pf, pt, c->dim, L.geo(P), u, f, out, diag, level_dw(c, 0), L.ih, s);
  } else {
    launch_gal(mode, pf, pt, c->dim, L.geo(P), u, f, out, level_st(c, l), level_dw(c, l), s);
  }
}

__global__ void k_zero_u4(int64_t n, uint4* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = uint4{0u, 0u, 0u, 0u};
}

// A fill kernel rather than a memset node, so that the cycle can be captured
// into a HIP graph; field sizes are multiples of 16 B (P % 4 == 0).
static void zero_field(helm_ctx* c, int l, int P, void* u, hipStream_t s) {
  const int64_t n = (int64_t)psize(field_prec(c, l)) * c->lv[l].npts * P / 16;
  if (c->plan) {
    Phase q{};
    q.op = PH_ZERO;
    q.out = u;
    q.n = n;
    c->plan->push_back(q);
    return;
  }
  hipLaunchKernelGGL(k_zero_u4, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, static_cast<uint4*>(u));
}

static void coarsest_solve(helm_ctx* c, int P, const void* f, void* out, hipStream_t s);
void field_axpy(helm_ctx* c, int l, int P, const void* x, void* y, hipStream_t s);

static void cycle_rec(helm_ctx* c, int l, int P, const void* f, void* out, void* tmp, hipStream_t s);

// K-cycle storage of coarse level l: v1, v2, w in the cycle's arithmetic
// precision, then per column the 3 x 2 Hessenberg matrix, the Gram
// coefficients, the least-squares solution and the norms.
static size_t kcycle_bytes(const helm_ctx* c, int l, int P) {
  const size_t vb = (psize(comp_prec(c)) * c->lv[l].npts * P + 255) / 256 * 256;
  return 3 * vb + 16 * (6 * (size_t)P + 6 * (size_t)P + 3 * (size_t)P + gram_part_elems(P) + 2 * (size_t)P) +
         8 * 3 * (size_t)P + 256;
}

// K-cycle coarse correction of level l (not the coarsest; the paper's
// K-FGMRES, section 5.3): the coarse problem M_l e = f (f in lv[l].F) is
// solved by two flexible GMRES steps from zero per column, each step
// preconditioned by the cycle of level l; e goes to lv[l].U0. The Krylov
// vectors are kept in the cycle's arithmetic precision (FP32 in mixed
// precision, where the level's fields are BF16); the preconditioned vectors
// z1, z2 are the cycle's outputs in the level's storage (U0 and kbuf).
static void kcycle_coarse(helm_ctx* c, int l, int P, hipStream_t s) {
  Level& L = c->lv[l];
  const int64_t N = L.npts;
  const Prec fp = field_prec(c, l), kp = comp_prec(c);
  char* m = c->klev[l];
  const size_t vb = (psize(kp) * N * P + 255) / 256 * 256;
  void* v1 = m;
  void* v2 = m + vb;
  void* w = m + 2 * vb;
  c128* Hm = reinterpret_cast<c128*>(m + 3 * vb);
  c128* Gc = Hm + 6 * (size_t)P;  // 2 (k+1) P entries, k = 2
  c128* Yc = Gc + 6 * (size_t)P;  // (k+1) P
  c128* part = Yc + 3 * (size_t)P;
  c128* Gs = part + gram_part_elems(P);
  double* b2 = reinterpret_cast<double*>(Gs + 2 * (size_t)P);
  double* hn2 = b2 + P;
  double* sc = hn2 + P;
  void* z[2] = {L.U0, c->kbuf[l]};
  // v1 = f / ||f|| (a zero column stays zero)
  const void* fin = L.F;
  if (fp != kp) {
    launch_convert(fp, kp, N * P, L.F, v1, s);
    fin = v1;
  }
  launch_colnorm2(kp, N, P, P, fin, part, Gs, b2, s);
  launch_inv_sqrt(P, b2, sc, s);
  launch_scale_cols(kp, N, P, P, sc, fin, v1, s);
  PtrList vl{};
  vl.p[0] = v1;
  vl.p[1] = v2;
  for (int j = 0; j < 2; ++j) {
    const void* vj = vl.p[j];
    // z_j = B v_j; the cycle reads its input in the level's storage (F is
    // free once v1 is formed)
    const void* cin = vj;
    if (fp != kp) {
      launch_convert(kp, fp, N * P, vj, L.F, s);
      cin = L.F;
    }
    cycle_rec(c, l, P, cin, z[j], L.U1, s);
    // w = M z_j, then one classical Gram-Schmidt pass against v_1..v_j
    if (fp != kp) {
      level_op(c, l, 0, P, z[j], nullptr, L.Rr, s);
      launch_convert(fp, kp, N * P, L.Rr, w, s);
    } else {
      level_op(c, l, 0, P, z[j], nullptr, w, s);
    }
    launch_gram(kp, N, P, P, 1, j + 1, vl, w, part, Gc, s);
    launch_update_norm(kp, N, P, P, j + 1, vl, Gc, w, part, Gs, hn2, s);
    launch_cg_hcol(P, j, 2, Gc, hn2, Hm, sc, s);
    if (j == 0) launch_scale_cols(kp, N, P, P, sc, w, v2, s);
  }
  // y = argmin || ||f|| e1 - H y || per column, e = z1 y1 + z2 y2 (into z1 = U0)
  launch_cg_ls(P, 2, Hm, b2, Gc, Yc, s);
  launch_kc_combine(fp, N, P, Yc, z[0], z[1], s);
}

// Multigrid cycle at level l for right-hand side f (level storage), result in
// `out`; `tmp` is a second buffer of the same size (ping-pong for Jacobi).
static void cycle_rec(helm_ctx* c, int l, int P, const void* f, void* out, void* tmp, hipStream_t s) {
  Level& L = c->lv[l];
  if (l == c->L - 1) {
    const bool was = c->prof;
    {
      Prof pr(c, HELM_K_COARSEST, s);
      c->prof = false;  // time the coarsest solve as one unit
      coarsest_solve(c, P, f, out, s);
      c->prof = was;
    }
    return;
  }
  const int npre = c->nu_pre[l], npost = c->nu_post[l];
  const int alternations = (npre >= 1 ? npre - 1 : 0) + npost;
  void* a = (alternations % 2 == 0) ? out : tmp;
  void* b = (a == out) ? tmp : out;
  Level& C = c->lv[l + 1];
  const Prec pf = field_prec(c, l), pc = field_prec(c, l + 1), pt = comp_prec(c);
  bool fused = false;
  if (npre == 2 && l == 0 && c->dim == 3 && !c->plan && can_pre_rr(pf, pc, pt, L.geo(P))) {
    // both pre-sweeps from a zero guess, the residual and the restriction in
    // one pass: b = JAC(w D^-1 f), C.F = R (f - M b)
    Prof pr(c, HELM_K_FINE_PRE_RR, s);
    const void* diag = c->precision == HELM_FP64 ? (const void*)L.dM : (const void*)L.dM32;
    fused = launch_pre_rr(pf, pc, pt, L.geo(P), C.geo(P), f, b, C.F, diag, level_dw(c, 0), L.ih, s);
    std::swap(a, b);
  } else if (npre >= 1) {
    int k1 = 1;
    if (l == 0 && c->dim == 3 && npre >= 2 && !c->plan && can_sweep01(pf, pt, L.geo(P))) {
      // the zero-guess sweep and the next one in one pass: b = JAC(w D^-1 f),
      // where the second sweep would have written
      Prof pr(c, HELM_K_FINE_SWEEP01, s);
      const void* diag = c->precision == HELM_FP64 ? (const void*)L.dM : (const void*)L.dM32;
      launch_sweep01(pf, pt, L.geo(P), f, b, diag, level_dw(c, 0), L.ih, s);
      std::swap(a, b);
      k1 = 2;
    } else {
      level_op(c, l, 3, P, nullptr, f, a, s);
    }
    for (int k = k1; k < npre; ++k) {
      level_op(c, l, 2, P, a, f, b, s);
      std::swap(a, b);
    }
  } else {
    zero_field(c, l, P, a, s);
  }
  if (!fused && l == 0 && c->dim == 3 && !c->plan && can_resid_restrict(pf, pc, pt, L.geo(P))) {
    // residual and restriction in one pass (counted as the fine residual)
    Prof pr(c, HELM_K_FINE_RESID, s);
    const void* diag = c->precision == HELM_FP64 ? (const void*)L.dM : (const void*)L.dM32;
    fused = launch_resid_restrict(pf, pc, pt, L.geo(P), C.geo(P), a, f, C.F, diag, L.ih, s);
  }
  if (!fused) {
    level_op(c, l, 1, P, a, f, L.Rr, s);
    if (c->plan) {
      Phase q{};
      q.op = PH_RESTRICT;
      q.pa = pf;
      q.pb = pc;
      q.g = L.geo(P);
      q.gc = C.geo(P);
      q.u = L.Rr;
      q.out = C.F;
      c->plan->push_back(q);
    } else {
      Prof pr(c, HELM_K_TRANSFER, s);
      launch_restrict(pf, pc, pt, c->dim, L.geo(P), C.geo(P), L.Rr, C.F, s);
    }
  }
  if (c->cycle == HELM_CYCLE_K && l + 1 < c->L - 1) {
    if (c->plan) c->plan_bad = true;  // the persistent cycle has no K-cycle
    kcycle_coarse(c, l + 1, P, s);
  } else {
    cycle_rec(c, l + 1, P, C.F, C.U0, C.U1, s);
  }
  if (c->cycle == HELM_CYCLE_W && l + 1 < c->L - 1) {
    if (c->plan) c->plan_bad = true;
    // W-cycle: a second coarse cycle on the residual of the first result,
    // e <- e + B(F - M e); F is free again and serves as ping-pong buffer.
    level_op(c, l + 1, 1, P, C.U0, C.F, c->kbuf[l + 1], s);
    cycle_rec(c, l + 1, P, c->kbuf[l + 1], C.U1, C.F, s);
    field_axpy(c, l + 1, P, C.U1, C.U0, s);
  }
  int k0 = 0;
  if (l == 0 && c->dim == 3 && npost >= 1 && !c->plan && can_prolong_sweep(pc, pf, pt, L.geo(P))) {
    // prolongation and correction fused into the first post-smoothing sweep:
    // b = JAC(a + P e); a itself is not updated (the next sweep overwrites it)
    Prof pr(c, HELM_K_FINE_PROSWEEP, s);
    const void* diag = c->precision == HELM_FP64 ? (const void*)L.dM : (const void*)L.dM32;
    if (launch_prolong_sweep(pc, pf, pt, L.geo(P), C.geo(P), C.U0, a, f, b, diag, level_dw(c, 0), L.ih, s)) {
      std::swap(a, b);
      k0 = 1;
    }
  }
  if (k0 == 0 && c->plan) {
    Phase q{};
    q.op = PH_PROLONG;
    q.pa = pc;
    q.pb = pf;
    q.g = L.geo(P);
    q.gc = C.geo(P);
    q.u = C.U0;
    q.out = a;
    c->plan->push_back(q);
  } else if (k0 == 0) {
    Prof pr(c, HELM_K_TRANSFER, s);
    launch_prolong_add(pc, pf, pt, c->dim, L.geo(P), C.geo(P), C.U0, a, s);
  }
  for (int k = k0; k < npost; ++k) {
    level_op(c, l, 2, P, a, f, b, s);
    std::swap(a, b);
  }
  (void)a;
}

// k steps of GMRES from zero on the coarsest grid, one independent GMRES per
// column (one classical Gram-Schmidt pass; the basis vectors after the first
// are normalised lazily, see launch_cg_lazy_coef), least squares by Givens
// rotations. No host synchronisation: the step count is fixed. `out` may be
// the buffer `f` (f is read only before the first step).
static void coarse_gmres(helm_ctx* c, int P, const void* f, void* out, int k, hipStream_t s) {
  const int l = c->L - 1;
  const Level& L = c->lv[l];
  const int64_t N = L.npts;
  const Prec p = field_prec(c, l);
  const size_t vb = (psize(p) * N * P + 255) / 256 * 256;
  char* m = static_cast<char*>(c->cg_mem);
  char* V = m;
  c128* H = reinterpret_cast<c128*>(m + vb * (k + 1));
  c128* Gc = H + (size_t)P * (k + 1) * k;
  c128* Yc = Gc + (size_t)2 * (k + 1) * P;
  c128* part = Yc + (size_t)(k + 1) * P;
  c128* Gs = part + gram_part_elems(P);
  double* b2 = reinterpret_cast<double*>(Gs + 2 * P);
  double* hn2 = b2 + P;
  double* sc = hn2 + P;
  double* nu = sc + P;  // (k + 1) P norms of the stored basis vectors
  auto vec = [&](int i) { return static_cast<void*>(V + vb * i); };
  launch_colnorm2(p, N, P, P, f, part, Gs, b2, s);
  launch_inv_sqrt(P, b2, sc, s);
  launch_scale_cols(p, N, P, P, sc, f, vec(0), s);
  launch_cg_lazy_init(P, b2, nu, s);
  PtrList vl{};
  for (int j = 0; j < k; ++j) {
    vl.p[j] = vec(j);
    level_op(c, l, 0, P, vec(j), nullptr, vec(j + 1), s);
    // one classical Gram-Schmidt pass; the update scales its output by
    // 1/nu_j and yields nu_{j+1}^2
    launch_gram(p, N, P, P, 1, j + 1, vl, vec(j + 1), part, Gc, s);
    launch_cg_lazy_coef(P, j, Gc, nu, sc, s);
    launch_update_norm(p, N, P, P, j + 1, vl, Gc, vec(j + 1), part, Gs, hn2, s, sc);
    launch_cg_lazy_hcol(P, j, k, Gc, hn2, nu, H, s);
  }
  launch_cg_ls(P, k, H, b2, Gc, Yc, s);  // Gc (2 (k+1) P entries) is free after the loop
  launch_lazy_y(P, k, nu, Yc, s);        // coefficients of the stored s_j = nu_j v_j
  launch_block_update(1, p, p, N, P, P, 1, k, vl, Yc, out, s);
}

// GMRES steps the coarsest storage must hold: coarse_iters, and for the
// learned correction at least the 20 steps of its fallback.
static int coarse_gmres_cap(const helm_ctx* c) {
  return c->coarse == HELM_COARSE_LEARNED ? std::max(c->coarse_iters, 20) : c->coarse_iters;
}

static size_t coarse_gmres_bytes(const helm_ctx* c, int P) {
  const int l = c->L - 1, k = coarse_gmres_cap(c);
  const size_t vb = (psize(field_prec(c, l)) * c->lv[l].npts * P + 255) / 256 * 256;
  return vb * (k + 1) + 16 * ((size_t)P * (k + 1) * k + 3 * (size_t)(k + 1) * P + gram_part_elems(P) + 2 * P) +
         8 * 3 * (size_t)P + 8 * (size_t)(k + 1) * P + 256;
}

static void coarsest_solve(helm_ctx* c, int P, const void* f, void* out, hipStream_t s) {
  const int l = c->L - 1;
  if (c->plan) {
    // the persistent cycle has the dense inverse (one GEMM) only
    if (c->coarse != HELM_COARSE_LU) {
      c->plan_bad = true;
      return;
    }
    Phase q{};
    q.op = PH_GEMM;
    q.pa = c->precision == HELM_FP64 ? P64 : P32;
    q.g.P = P;
    q.n = c->nc;
    q.u = f;
    q.out = out;
    q.c0 = c->precision == HELM_FP64 ? (const void*)c->Minv64 : (const void*)c->Minv32;
    c->plan->push_back(q);
    return;
  }
  if (c->coarse == HELM_COARSE_LU) {
    if (c->precision == HELM_FP64)
      launch_gemm(P64, c->nc, P, c->nc, c128{1, 0}, c->Minv64, c->nc, f, P, c128{0, 0}, out, P, s);
    else
      launch_gemm(P32, c->nc, P, c->nc, c128{1, 0}, c->Minv32, c->nc, f, P, c128{0, 0}, out, P, s);
  } else if (c->coarse == HELM_COARSE_GMRES) {
    // restarted GMRES(coarse_iters): the first cycle from zero, each further
    // one on the current residual (Rr of the coarsest level is free)
    coarse_gmres(c, P, f, out, c->coarse_iters, s);
    for (int q = 1; q < c->coarse_restarts; ++q) {
      void* r = c->lv[l].Rr;
      level_op(c, l, 1, P, out, f, r, s);
      coarse_gmres(c, P, r, r, c->coarse_iters, s);
      field_axpy(c, l, P, r, out, s);
    }
  } else if (c->coarse == HELM_COARSE_LEARNED && c->net) {
    bool ok = false;
    if (c->capturing) {
      // inside a graph: no host check here; the caller reads the network's
      // non-finite count after the replay and redoes the cycle if needed
      learned::apply_async(c->net, P, f, out, s);
      ok = true;
    } else if (!c->force_fallback && !c->rate_fallback) {
      ok = learned::apply(c->net, P, f, out, s);
    }
    if (!ok) {
      ++c->fallbacks;
      coarse_gmres(c, P, f, out, coarse_gmres_cap(c), s);
    } else if (c->coarse_iters > 0) {
      // the network's correction is the initial guess of restarted
      // GMRES(coarse_iters) on the remaining residual (Rr of the coarsest
      // level is free)
      void* r = c->lv[l].Rr;
      for (int q = 0; q < c->coarse_restarts; ++q) {
        level_op(c, l, 1, P, out, f, r, s);
        coarse_gmres(c, P, r, r, c->coarse_iters, s);
        field_axpy(c, l, P, r, out, s);
      }
    }
  } else {
    // relaxation only: nu_pre + nu_post damped Jacobi sweeps from zero
    const int sweeps = std::max(1, c->nu_pre[l] + c->nu_post[l]);
    void* tmp = c->lv[l].U1 == out ? c->lv[l].Rr : c->lv[l].U1;
    void* a = (sweeps - 1) % 2 == 0 ? out : tmp;
    void* b = a == out ? tmp : out;
    level_op(c, l, 3, P, nullptr, f, a, s);
    for (int k = 1; k < sweeps; ++k) {
      level_op(c, l, 2, P, a, f, b, s);
      std::swap(a, b);
    }
  }
  // training pairs for the learned correction (exact or GMRES solves only)
  if (c->cap && (c->coarse == HELM_COARSE_LU || c->coarse == HELM_COARSE_GMRES)) learned::capture(c->cap, P, f, out, s);
}

static void clear_graphs(helm_ctx* c) {
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  c->graphs.clear();
  for (auto& p : c->plans) (void)hipFree(p.d);
  c->plans.clear();
}

// One cycle f -> out as one cooperative launch of the persistent kernel. The
// cycle's launches are recorded once per (block width, buffers) as phases
// (the generic kernels' work items; the fused 3D forms are left out) and
// copied to the device.
static helm_status run_persist(helm_ctx* c, int P, const void* f, void* out, void* tmp, hipStream_t s) {
  helm_ctx::CyclePlan* pl = nullptr;
  for (auto& q : c->plans)
    if (q.P == P && q.f == f && q.out == out && q.tmp == tmp) pl = &q;
  if (!pl) {
    std::vector<Phase> ph;
    c->plan = &ph;
    c->plan_bad = false;
    cycle_rec(c, 0, P, f, out, tmp, s);
    c->plan = nullptr;
    if (c->plan_bad)
      return fail(HELM_ERR_INVALID_ARG, "the persistent cycle needs a V-cycle with the LU coarsest solver");
    const bool mixed = c->precision != HELM_FP64;
    const int gmax = persist_grid(c->dim, mixed);
    if (gmax < 1) return fail(HELM_ERR_DEVICE, "the device cannot run the cooperative cycle kernel");
    int64_t need = 1;  // workgroups the widest phase can use
    auto cols = [](int p) { return p == P64 ? 1 : (p == P32 ? 2 : 4); };  // columns per 16-byte unit
    for (const Phase& q : ph) {
      int64_t items = 0;
      const int k2 = std::max(cols(q.pa), cols(q.pb));
      if (q.op == PH_FINE || q.op == PH_GAL) items = q.g.npts * q.g.P / cols(q.pa);
      else if (q.op == PH_PROLONG) items = q.g.npts * q.g.P / k2;
      else if (q.op == PH_RESTRICT) items = q.gc.npts * q.gc.P / k2;
      else if (q.op == PH_ZERO) items = q.n;
      else if (q.op == PH_GEMM) items = 256 * ((q.n + 63) / 64) * ((q.g.P + 63) / 64);
      need = std::max(need, (items + 255) / 256);
    }
    helm_ctx::CyclePlan np{P, f, out, tmp, nullptr, (int)ph.size(), (int)std::min<int64_t>(need, gmax)};
    HCHECK(dmalloc(&np.d, sizeof(Phase) * ph.size()));
    const hipError_t e = hipMemcpy(np.d, ph.data(), sizeof(Phase) * ph.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(np.d);
      HCHECK(e);
    }
    c->plans.push_back(np);
    pl = &c->plans.back();
  }
  HCHECK(launch_cycle_persist(c->dim, c->precision != HELM_FP64, pl->d, pl->nph, pl->grid, s));
  return HELM_OK;
}

// One cycle f -> out on level 0: eager launches (form 0), a HIP graph
// (form 1) or the persistent kernel (form 2). With a graph, the kernel sequence of this
// (block width, buffers) is captured once into a HIP graph on a private
// stream and replayed on s afterwards; the cycle has no host synchronisation
// or memset inside, so the replay runs exactly the kernels of the eager path.
// The learned correction's non-finite check happens after the replay: if it
// fired, the cycle is run again eagerly with the GMRES fallback.
static helm_status run_cycle(helm_ctx* c, int P, const void* f, void* out, void* tmp, int form, hipStream_t s) {
  if (form == 2) return run_persist(c, P, f, out, tmp, s);
  if (form != 1) {
    cycle_rec(c, 0, P, f, out, tmp, s);
    return HELM_OK;
  }
  const bool net = c->coarse == HELM_COARSE_LEARNED && c->net;
  if (net) {
    helm_status st = learned::prepare(c->net, P);
    if (st != HELM_OK) return st;
    if (learned::scratch_gen(c->net) != c->graph_net_gen) {
      clear_graphs(c);
      c->graph_net_gen = learned::scratch_gen(c->net);
    }
  }
  hipGraphExec_t exec = nullptr;
  for (const auto& g : c->graphs)
    if (g.P == P && g.f == f && g.out == out && g.tmp == tmp) exec = g.exec;
  if (!exec) {
    if (c->graphs.size() >= 64) clear_graphs(c);
    if (!c->gstream) HCHECK(hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
    HCHECK(hipStreamBeginCapture(c->gstream, hipStreamCaptureModeRelaxed));
    c->capturing = true;
    cycle_rec(c, 0, P, f, out, tmp, c->gstream);
    c->capturing = false;
    hipGraph_t g = nullptr;
    HCHECK(hipStreamEndCapture(c->gstream, &g));
    const hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HCHECK(e);
    c->graphs.push_back({P, f, out, tmp, exec});
  }
  HCHECK(hipGraphLaunch(exec, s));
  if (net) {
    const int bad = learned::bad_count(c->net, s);
    if (bad < 0) return fail(HELM_ERR_DEVICE, "reading the network's non-finite count failed");
    if (bad > 0) {
      c->force_fallback = true;
      cycle_rec(c, 0, P, f, out, tmp, s);
      c->force_fallback = false;
    }
  }
  return HELM_OK;
}

static learned::Coarse coarse_view(const helm_ctx* c) {
  const Level& L = c->lv[c->L - 1];
  learned::Coarse g;
  for (int a = 0; a < 3; ++a) g.nu[a] = L.nu[a];
  g.H2 = L.h[0] * L.h[0];
  g.p = field_prec(c, c->L - 1);
  g.st = L.st64;
  return g;
}

}  // namespace helm

// ---------------------------------------------------------------------------
// Field allocation for a block of P columns.
// ---------------------------------------------------------------------------
static int padP(int nrhs) { return (nrhs + 3) / 4 * 4; }

static helm_status ensure_fields(helm_ctx* c, int P) {
  if (c->fieldsP >= P && c->fieldmem) return HELM_OK;
  clear_graphs(c);
  if (c->fieldmem) {
    hipFree(c->fieldmem);
    c->fieldmem = nullptr;
  }
  size_t total = 0;
  for (int l = 0; l < c->L; ++l) total += 5 * ((psize(field_prec(c, l)) * c->lv[l].npts * P + 255) / 256 * 256);
  HCHECK(dmalloc(&c->fieldmem, total));
  char* p = static_cast<char*>(c->fieldmem);
  c->kbuf.assign(c->L, nullptr);
  for (int l = 0; l < c->L; ++l) {
    const size_t b = (psize(field_prec(c, l)) * c->lv[l].npts * P + 255) / 256 * 256;
    c->lv[l].F = p;
    c->lv[l].U0 = p + b;
    c->lv[l].U1 = p + 2 * b;
    c->lv[l].Rr = p + 3 * b;
    c->kbuf[l] = p + 4 * b;
    p += 5 * b;
  }
  if (c->coarse == HELM_COARSE_GMRES || c->coarse == HELM_COARSE_LEARNED) {
    hipFree(c->cg_mem);
    c->cg_mem = nullptr;
    HCHECK(dmalloc(&c->cg_mem, coarse_gmres_bytes(c, P)));
  }
  hipFree(c->kmem);
  c->kmem = nullptr;
  c->klev.assign(c->L, nullptr);
  if (c->cycle == HELM_CYCLE_K && c->L > 2) {
    size_t kt = 0;
    for (int l = 1; l < c->L - 1; ++l) kt += kcycle_bytes(c, l, P);
    HCHECK(dmalloc(&c->kmem, kt));
    char* q = static_cast<char*>(c->kmem);
    for (int l = 1; l < c->L - 1; ++l) {
      c->klev[l] = q;
      q += kcycle_bytes(c, l, P);
    }
  }
  c->fieldsP = P;
  return HELM_OK;
}

// ---------------------------------------------------------------------------
// Autotuner for the finest-level marching kernel: times each candidate tile
// (rows per lane x planes per chunk) on the real buffers with HIP events and
// keeps the fastest. Choices are cached in a JSON-lines file named by the
// HELM_TUNE_CACHE environment variable, keyed by arch, grid, block width and
// precision; HELM_AUTOTUNE=0 keeps the default tile.
// ---------------------------------------------------------------------------
static std::string tune_key(const helm_ctx* c, int P) {
  char b[160];
  std::snprintf(b, sizeof(b), "gfx950:%d:%d:%d:%d:%s", c->lv[0].nu[0], c->lv[0].nu[1], c->lv[0].nu[2], P,
                c->precision == HELM_FP64 ? "fp64" : "mixed");
  return b;
}

static bool tune_cache_lookup(const std::string& key, FineTile* t) {
  const char* path = std::getenv("HELM_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE* fp = std::fopen(path, "r");
  if (!fp) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof(line), fp)) {
    char k[200];
    int ry, zc;
    if (std::sscanf(line, " {\"key\": \"%199[^\"]\", \"ry\": %d, \"zc\": %d", k, &ry, &zc) == 3 && key == k &&
        (ry == 1 || ry == 2 || ry == 4 || ry == 8 || ry == 16) && zc > 0) {
      *t = FineTile{ry, zc};
      found = true;  // the last entry for a key wins
    }
  }
  std::fclose(fp);
  return found;
}

static void tune_cache_store(const std::string& key, FineTile t, double ms) {
  const char* path = std::getenv("HELM_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* fp = std::fopen(path, "a");
  if (!fp) return;
  std::fprintf(fp, "{\"key\": \"%s\", \"ry\": %d, \"zc\": %d, \"ms\": %.4f}\n", key.c_str(), t.ry, t.zc, ms);
  std::fclose(fp);
}

static helm_status autotune_fine(helm_ctx* c, int P, hipStream_t s) {
  if (c->dim != 3 || c->tileP == P) return HELM_OK;
  clear_graphs(c);  // captured cycles hold the previous tile's kernels
  c->tileP = P;
  c->tile = FineTile{4, 32};
  const char* en = std::getenv("HELM_AUTOTUNE");
  if (en && std::strcmp(en, "0") == 0) return HELM_OK;
  const std::string key = tune_key(c, P);
  FineTile t;
  if (tune_cache_lookup(key, &t)) {
    c->tile = t;
    return HELM_OK;
  }
  // Each candidate is timed on a whole cycle (the fused finest-level kernels
  // exist for some tiles only, and the LDS tiles also select the LDS form of
  // the Galerkin sweeps), from a zero right-hand side in the level-0 buffers,
  // with kernel timing and pair capture off.
  Level& L = c->lv[0];
  const size_t bytes = psize(field_prec(c, 0)) * L.npts * P;
  HCHECK(hipMemsetAsync(L.F, 0, bytes, s));
  hipEvent_t a, b;
  HCHECK(hipEventCreate(&a));
  HCHECK(hipEventCreate(&b));
  // rows per lane of the register-blocked kernel, or 8 / 16: the LDS-blocked
  // kernel on 16 x 8 / 16 x 16 tiles (k_fine_t16)
  const int rys[5] = {1, 2, 4, 8, 16};
  const int zcs[4] = {16, 24, 32, 64};
  double best = 1e30;
  FineTile bt = c->tile;
  const bool was = c->prof;
  learned::Net* cap = c->cap;
  const int64_t fb0 = c->fallbacks;
  c->prof = false;
  c->cap = nullptr;
  for (int ri = 0; ri < 5; ++ri)
    for (int zi = 0; zi < 4; ++zi) {
      set_fine_tile(FineTile{rys[ri], zcs[zi]});
      cycle_rec(c, 0, P, L.F, L.U0, L.U1, s);  // warm-up
      std::vector<float> ts;
      for (int r = 0; r < 3; ++r) {
        hipEventRecord(a, s);
        cycle_rec(c, 0, P, L.F, L.U0, L.U1, s);
        hipEventRecord(b, s);
        hipEventSynchronize(b);
        float ms = 0.f;
        hipEventElapsedTime(&ms, a, b);
        ts.push_back(ms);
      }
      std::sort(ts.begin(), ts.end());
      if (ts[1] < best) {
        best = ts[1];
        bt = FineTile{rys[ri], zcs[zi]};
      }
    }
  c->prof = was;
  c->cap = cap;
  c->fallbacks = fb0;
  hipEventDestroy(a);
  hipEventDestroy(b);
  HCHECK(hipGetLastError());
  c->tile = bt;
  tune_cache_store(key, bt, best);
  return HELM_OK;
}

namespace helm {

__global__ void k_field_axpy_c128(int64_t n, const c128* x, c128* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = c128{y[i].re + x[i].re, y[i].im + x[i].im};
}
__global__ void k_field_axpy_c64(int64_t n, const c64* x, c64* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = c64{y[i].re + x[i].re, y[i].im + x[i].im};
}
__global__ void k_field_axpy_cbf(int64_t n, const cbf* x, cbf* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n)
    y[i] = cbf{f2bf(bf2f(y[i].re) + bf2f(x[i].re)), f2bf(bf2f(y[i].im) + bf2f(x[i].im))};
}

void field_axpy(helm_ctx* c, int l, int P, const void* x, void* y, hipStream_t s) {
  const int64_t n = c->lv[l].npts * P;
  const dim3 gr((unsigned)((n + 255) / 256));
  switch (field_prec(c, l)) {
    case P64: hipLaunchKernelGGL(k_field_axpy_c128, gr, dim3(256), 0, s, n, (const c128*)x, (c128*)y); break;
    case P32: hipLaunchKernelGGL(k_field_axpy_c64, gr, dim3(256), 0, s, n, (const c64*)x, (c64*)y); break;
    default: hipLaunchKernelGGL(k_field_axpy_cbf, gr, dim3(256), 0, s, n, (const cbf*)x, (cbf*)y); break;
  }
}

}  // namespace helm

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------
extern "C" {

void helm_setup_desc_default(helm_setup_desc* d) {
  std::memset(d, 0, sizeof(*d));
  d->dim = 3;
  d->shift = 0.2;
  d->levels = 3;
  for (int l = 0; l < HELM_MAX_LEVELS; ++l) {
    d->nu_pre[l] = 2;
    d->nu_post[l] = 2;
    d->jacobi_weight[l] = 0.8;
  }
  d->precision = HELM_FP64;
  d->coarse = HELM_COARSE_LU;
  d->cycle = HELM_CYCLE_V;
  d->coarse_iters = 20;
  d->coarse_restarts = 1;
}

const char* helm_status_string(helm_status s) {
  switch (s) {
    case HELM_OK: return "ok";
    case HELM_ERR_INVALID_ARG: return "invalid argument";
    case HELM_ERR_OOM: return "out of device memory";
    case HELM_ERR_DEVICE: return "device error";
    case HELM_ERR_NOT_CONVERGED: return "not converged";
    case HELM_ERR_BREAKDOWN: return "block breakdown";
    case HELM_ERR_NONFINITE: return "non-finite input";
    case HELM_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown";
}

const char* helm_last_error(void) { return g_err.c_str(); }

static void cap_detach(helm_ctx* h);

static void free_ctx(helm_ctx* c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  cap_detach(c);
  clear_graphs(c);
  if (c->gstream) (void)hipStreamDestroy(c->gstream);
  if (c->bstream) (void)hipStreamDestroy(c->bstream);
  for (int l = 0; l < c->L; ++l) {
    Level& L = c->lv[l];
    hipFree(L.dH);
    hipFree(L.dM);
    hipFree(L.dS);
    hipFree(L.dw64);
    hipFree(L.dM32);
    hipFree(L.dw32);
    hipFree(L.st64);
    hipFree(L.st32);
  }
  hipFree(c->Minv64);
  hipFree(c->Minv32);
  hipFree(c->fieldmem);
  hipFree(c->kmem);
  hipFree(c->cg_mem);
  hipFree(c->ws);
  hipFree(c->resid_buf);
  hipFree(c->sensbuf);
  if (c->hbuf) hipHostFree(c->hbuf);
  if (c->net) learned::destroy(c->net);
  for (hipEvent_t e : c->evpool) hipEventDestroy(e);
  delete c;
}

void helm_destroy(helm_handle h) { free_ctx(h); }

helm_status helm_setup(const helm_setup_desc* d, void* stream, helm_handle* out) {
  if (!d || !out) return fail(HELM_ERR_INVALID_ARG, "null descriptor or output");
  *out = nullptr;
  if (d->dim != 2 && d->dim != 3) return fail(HELM_ERR_INVALID_ARG, "dim must be 2 or 3");
  if (d->levels < 2 || d->levels > HELM_MAX_LEVELS) return fail(HELM_ERR_INVALID_ARG, "levels must be 2..%d", HELM_MAX_LEVELS);
  if (!(d->omega > 0) || !(d->shift >= 0) || !std::isfinite(d->omega) || !std::isfinite(d->shift))
    return fail(HELM_ERR_INVALID_ARG, "omega must be > 0 and shift >= 0");
  if (d->precision != HELM_FP64 && d->precision != HELM_MIXED) return fail(HELM_ERR_INVALID_ARG, "bad precision");
  if (d->coarse < HELM_COARSE_LU || d->coarse > HELM_COARSE_GMRES) return fail(HELM_ERR_INVALID_ARG, "bad coarse kind");
  // the coarsest GMRES keeps its basis vectors in one PtrList (MAXPTR slots)
  if (d->coarse == HELM_COARSE_GMRES && (d->coarse_iters < 1 || d->coarse_iters > MAXPTR))
    return fail(HELM_ERR_INVALID_ARG, "coarse_iters must be 1..%d", MAXPTR);
  if (d->coarse == HELM_COARSE_LEARNED && (d->coarse_iters < 0 || d->coarse_iters > MAXPTR))
    return fail(HELM_ERR_INVALID_ARG, "coarse_iters must be 0..%d with the learned coarsest correction", MAXPTR);
  if (d->coarse_restarts < 0 || d->coarse_restarts > 16)
    return fail(HELM_ERR_INVALID_ARG, "coarse_restarts must be 0..16 (0 and 1: one GMRES cycle)");
  if (d->cycle < HELM_CYCLE_V || d->cycle > HELM_CYCLE_K) return fail(HELM_ERR_INVALID_ARG, "bad cycle kind");
  const int f = 1 << (d->levels - 1);
  int64_t N = 1;
  for (int a = 0; a < d->dim; ++a) {
    if (d->n[a] < 2 * f || d->n[a] % f != 0)
      return fail(HELM_ERR_INVALID_ARG, "n[%d]=%d must be a multiple of 2^(levels-1)=%d with >= 1 coarsest unknown", a,
                  d->n[a], f);
    if (!(d->h[a] > 0)) return fail(HELM_ERR_INVALID_ARG, "h[%d] must be > 0", a);
    N *= d->n[a] - 1;
  }
  for (int l = 0; l < d->levels; ++l)
    if (d->nu_pre[l] < 0 || d->nu_post[l] < 0 || !std::isfinite(d->jacobi_weight[l]))
      return fail(HELM_ERR_INVALID_ARG, "bad relaxation parameters at level %d", l);
  if (!d->m || !d->gamma) return fail(HELM_ERR_INVALID_ARG, "m and gamma are required");
  for (int64_t i = 0; i < N; ++i) {
    if (!std::isfinite(d->m[i]) || !std::isfinite(d->gamma[i]))
      return fail(HELM_ERR_NONFINITE, "non-finite m or gamma at %lld", (long long)i);
    if (!(d->m[i] > 0) || d->gamma[i] < 0) return fail(HELM_ERR_INVALID_ARG, "m must be > 0 and gamma >= 0");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  helm_ctx* c = new helm_ctx();
  c->dim = d->dim;
  c->L = d->levels;
  c->precision = d->precision;
  c->coarse = d->coarse;
  c->cycle = d->cycle;
  c->coarse_iters = d->coarse_iters;
  c->coarse_restarts = std::max(1, d->coarse_restarts);
  c->omega = d->omega;
  c->shift = d->shift;
  for (int l = 0; l < HELM_MAX_LEVELS; ++l) {
    c->nu_pre[l] = d->nu_pre[l];
    c->nu_post[l] = d->nu_post[l];
    c->wj[l] = d->jacobi_weight[l];
  }
  helm_status st = HELM_OK;
  auto bail = [&](helm_status e) {
    free_ctx(c);
    return e;
  };
  // geometry per level
  for (int l = 0; l < c->L; ++l) {
    Level& L = c->lv[l];
    L.npts = 1;
    for (int a = 0; a < 3; ++a) {
      if (a < c->dim) {
        const int cells = d->n[a] >> l;
        L.nu[a] = cells - 1;
        L.h[a] = d->h[a] * (double)(1 << l);
        L.ih[a] = 1.0 / (L.h[a] * L.h[a]);
      } else {
        L.nu[a] = 1;
        L.h[a] = 1.0;
        L.ih[a] = 0.0;
      }
      L.npts *= L.nu[a];
    }
    L.pf = field_prec(c, l);
  }
  const int NS = c->dim == 3 ? 27 : 9;
  // fine coefficients
  {
    Level& L = c->lv[0];
    double *dm = nullptr, *dg = nullptr;
    if (dmalloc(&dm, 8 * N) != hipSuccess || dmalloc(&dg, 8 * N) != hipSuccess ||
        dmalloc(&L.dH, 16 * N) != hipSuccess || dmalloc(&L.dM, 16 * N) != hipSuccess ||
        dmalloc(&L.dw64, 16 * N) != hipSuccess || dmalloc(&L.dS, 16 * N) != hipSuccess) {
      hipFree(dm);
      hipFree(dg);
      return bail(fail(HELM_ERR_OOM, "setup: fine coefficients"));
    }
    hipMemcpyAsync(dm, d->m, 8 * N, hipMemcpyHostToDevice, s);
    hipMemcpyAsync(dg, d->gamma, 8 * N, hipMemcpyHostToDevice, s);
    launch_fine_coef(c->dim, N, dm, dg, c->omega, c->shift, c->wj[0], L.ih, L.dH, L.dM, L.dw64, s);
    launch_sens_coef(N, dg, c->omega, L.dS, s);
    hipStreamSynchronize(s);
    hipFree(dm);
    hipFree(dg);
    if (c->precision == HELM_MIXED) {
      if (dmalloc(&L.dM32, 8 * N) != hipSuccess || dmalloc(&L.dw32, 8 * N) != hipSuccess)
        return bail(fail(HELM_ERR_OOM, "setup: fine FP32 coefficients"));
      launch_narrow(N, L.dM, L.dM32, s);
      launch_narrow(N, L.dw64, L.dw32, s);
    }
  }
  // Galerkin levels
  for (int l = 1; l < c->L; ++l) {
    Level& L = c->lv[l];
    Level& F = c->lv[l - 1];
    if (dmalloc(&L.st64, 16 * L.npts * NS) != hipSuccess || dmalloc(&L.dw64, 16 * L.npts) != hipSuccess)
      return bail(fail(HELM_ERR_OOM, "setup: level %d stencil", l));
    if (l == 1)
      launch_galerkin_from_fine(c->dim, F.geo(4), L.geo(4), F.dM, F.ih, L.st64, s);
    else
      launch_galerkin_from_gal(c->dim, F.geo(4), L.geo(4), F.st64, L.st64, s);
    launch_gal_dw(c->dim, L.npts, L.st64, c->wj[l], L.dw64, s);
    if (c->precision == HELM_MIXED) {
      if (dmalloc(&L.st32, 8 * L.npts * NS) != hipSuccess || dmalloc(&L.dw32, 8 * L.npts) != hipSuccess)
        return bail(fail(HELM_ERR_OOM, "setup: level %d FP32 stencil", l));
      launch_narrow(L.npts * NS, L.st64, L.st32, s);
      launch_narrow(L.npts, L.dw64, L.dw32, s);
    }
  }
  if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess)
    return bail(fail(HELM_ERR_DEVICE, "setup: hierarchy kernels failed"));
  // coarsest dense inverse
  c->nc = c->lv[c->L - 1].npts;
  if (c->coarse == HELM_COARSE_LU) {
    const int64_t n = c->nc;
    if (n > 32768) return bail(fail(HELM_ERR_UNSUPPORTED, "coarsest grid has %lld unknowns (> 32768)", (long long)n));
    const int nb = 32;  // pivot block held in LDS by one workgroup
    c128* work = nullptr;
    if (dmalloc(&c->Minv64, 16 * n * n) != hipSuccess ||
        dmalloc(&work, 16 * (2 * n * nb + nb * nb + 1)) != hipSuccess) {
      hipFree(work);
      return bail(fail(HELM_ERR_OOM, "setup: coarsest inverse (%lld unknowns)", (long long)n));
    }
    launch_assemble_dense(c->dim, c->lv[c->L - 1].geo(4), c->lv[c->L - 1].st64, c->Minv64, s);
    const int rc = gauss_jordan_inverse(n, c->Minv64, nb, work, s);
    hipFree(work);
    if (rc != 0) return bail(fail(HELM_ERR_DEVICE, "setup: coarsest inversion failed (%d)", rc));
    if (c->precision == HELM_MIXED) {
      if (dmalloc(&c->Minv32, 8 * n * n) != hipSuccess) return bail(fail(HELM_ERR_OOM, "setup: FP32 coarsest inverse"));
      launch_narrow(n * n, c->Minv64, c->Minv32, s);
      hipStreamSynchronize(s);
      hipFree(c->Minv64);
      c->Minv64 = nullptr;
    }
  } else if (c->coarse == HELM_COARSE_LEARNED) {
    if (c->dim != 3) return bail(fail(HELM_ERR_UNSUPPORTED, "the learned coarsest correction is 3D only"));
    std::vector<float> prm(learned::nparams());
    if ((st = learned::read_blob(d->net, d->net_bytes, prm.data())) != HELM_OK) return bail(st);
    const learned::Coarse g = coarse_view(c);
    const int D = learned::edge_for(g);
    // samples per network pass: bounded activation memory (about 270 B per voxel)
    const int64_t V = (int64_t)D * D * D;
    const int bmax = (int)std::max<int64_t>(1, std::min<int64_t>(64, (int64_t)(4LL << 30) / (272 * V)));
    if ((st = learned::create(D, bmax, 0, s, &c->net)) != HELM_OK) return bail(st);
    if ((st = learned::set_params(c->net, prm.data(), s)) != HELM_OK) return bail(st);
    if ((st = learned::bind(c->net, g, s)) != HELM_OK) return bail(st);
  }
  if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess)
    return bail(fail(HELM_ERR_DEVICE, "setup: device error"));
  *out = c;
  return HELM_OK;
}

helm_status helm_profile_enable(helm_handle h, int32_t enable) {
  if (!h) return fail(HELM_ERR_INVALID_ARG, "null handle");
  HCHECK(hipDeviceSynchronize());
  h->prof = enable != 0;
  if (h->prof) {
    h->evused = 0;
    h->evcls.clear();
  }
  return HELM_OK;
}

helm_status helm_profile_read(helm_handle h, helm_kernel_stat* stats) {
  if (!h || !stats) return fail(HELM_ERR_INVALID_ARG, "null argument");
  HCHECK(hipDeviceSynchronize());
  for (int k = 0; k < HELM_K_NCLASS; ++k) stats[k] = helm_kernel_stat{0, 0.0};
  for (size_t p = 0; p < h->evcls.size(); ++p) {
    float ms = 0.f;
    HCHECK(hipEventElapsedTime(&ms, h->evpool[2 * p], h->evpool[2 * p + 1]));
    const int cls = h->evcls[p];
    if (cls >= 0 && cls < HELM_K_NCLASS) {
      stats[cls].launches += 1;
      stats[cls].total_ms += ms;
    }
  }
  return HELM_OK;
}

helm_status helm_fine_tile(helm_handle h, int32_t nrhs, int32_t tile[2]) {
  if (!h || !tile || nrhs < 1 || nrhs > 256) return fail(HELM_ERR_INVALID_ARG, "bad argument");
  const int P = padP(nrhs);
  helm_status st;
  if ((st = ensure_fields(h, P)) != HELM_OK) return st;
  if ((st = autotune_fine(h, P, nullptr)) != HELM_OK) return st;
  tile[0] = h->tile.ry;
  tile[1] = h->tile.zc;
  return HELM_OK;
}

helm_status helm_set_fine_tile(helm_handle h, int32_t nrhs, const int32_t tile[2]) {
  if (!h || !tile || nrhs < 1 || nrhs > 256) return fail(HELM_ERR_INVALID_ARG, "bad argument");
  if (!(tile[0] == 1 || tile[0] == 2 || tile[0] == 4 || tile[0] == 8 || tile[0] == 16) || tile[1] < 1)
    return fail(HELM_ERR_INVALID_ARG, "bad tile");
  clear_graphs(h);
  h->tileP = padP(nrhs);
  h->tile = FineTile{tile[0], tile[1]};
  return HELM_OK;
}

helm_status helm_level_dims(helm_handle h, int32_t level, int32_t nu[3]) {
  if (!h || !nu || level < 0 || level >= h->L) return fail(HELM_ERR_INVALID_ARG, "bad level");
  for (int a = 0; a < 3; ++a) nu[a] = h->lv[level].nu[a];
  return HELM_OK;
}

helm_status helm_level_stencil(helm_handle h, int32_t level, double* st) {
  if (!h || !st || level < 1 || level >= h->L) return fail(HELM_ERR_INVALID_ARG, "bad level");
  const int NS = h->dim == 3 ? 27 : 9;
  HCHECK(hipDeviceSynchronize());
  HCHECK(hipMemcpy(st, h->lv[level].st64, 16 * h->lv[level].npts * NS, hipMemcpyDeviceToHost));
  return HELM_OK;
}


static helm_status check_block(helm_handle h, int32_t nrhs, const void* a, const void* b) {
  if (!h) return fail(HELM_ERR_INVALID_ARG, "null handle");
  if (nrhs < 1 || nrhs > 256) return fail(HELM_ERR_INVALID_ARG, "nrhs must be 1..256");
  if (!a || !b) return fail(HELM_ERR_INVALID_ARG, "null device pointer");
  return HELM_OK;
}

// Scratch for the ABI helpers: internal copies of two blocks.
static helm_status tmp_blocks(helm_ctx* c, int P, int64_t N, c128** A, c128** B) {
  HCHECK(dmalloc(A, 16 * N * P));
  if (dmalloc(B, 16 * N * P) != hipSuccess) {
    hipFree(*A);
    return fail(HELM_ERR_OOM, "temporary block");
  }
  (void)c;
  return HELM_OK;
}

helm_status helm_apply(helm_handle h, int32_t op, int32_t nrhs, const void* X, void* Y, void* stream) {
  helm_status st = check_block(h, nrhs, X, Y);
  if (st != HELM_OK) return st;
  if (op != 0 && op != 1) return fail(HELM_ERR_INVALID_ARG, "op must be 0 (H) or 1 (M)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int P = padP(nrhs);
  const Level& L = h->lv[0];
  c128 *A, *B;
  if ((st = tmp_blocks(h, P, L.npts, &A, &B)) != HELM_OK) return st;
  launch_to_internal(P64, L.npts, nrhs, P, X, A, s);
  launch_fine(0, P64, P64, P64, P64, h->dim, L.geo(P), A, nullptr, B, op == 0 ? L.dH : L.dM, nullptr, L.ih, s);
  launch_to_abi(P64, L.npts, nrhs, P, B, Y, s);
  hipError_t e = hipStreamSynchronize(s);
  hipFree(A);
  hipFree(B);
  HCHECK(e);
  HCHECK(hipGetLastError());
  return HELM_OK;
}

helm_status helm_precond(helm_handle h, int32_t nrhs, const void* R, void* Z, void* stream) {
  helm_status st = check_block(h, nrhs, R, Z);
  if (st != HELM_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int P = padP(nrhs);
  if ((st = ensure_fields(h, P)) != HELM_OK) return st;
  set_fine_tile(h->tileP == P ? h->tile : FineTile{4, 32});
  Level& L = h->lv[0];
  const Prec pf = field_prec(h, 0);
  c128 *A, *B;
  if ((st = tmp_blocks(h, P, L.npts, &A, &B)) != HELM_OK) return st;
  launch_to_internal(pf, L.npts, nrhs, P, R, L.F, s);
  cycle_rec(h, 0, P, L.F, A, B, s);
  launch_to_abi(pf, L.npts, nrhs, P, A, Z, s);
  hipError_t e = hipStreamSynchronize(s);
  hipFree(A);
  hipFree(B);
  HCHECK(e);
  HCHECK(hipGetLastError());
  return HELM_OK;
}

helm_status helm_coarse_solve(helm_handle h, int32_t nrhs, const void* R, void* E, void* stream) {
  helm_status st = check_block(h, nrhs, R, E);
  if (st != HELM_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int P = padP(nrhs);
  if ((st = ensure_fields(h, P)) != HELM_OK) return st;
  const int l = h->L - 1;
  Level& L = h->lv[l];
  const Prec pf = field_prec(h, l);
  launch_to_internal(pf, L.npts, nrhs, P, R, L.F, s);
  coarsest_solve(h, P, L.F, L.U0, s);
  launch_to_abi(pf, L.npts, nrhs, P, L.U0, E, s);
  HCHECK(hipStreamSynchronize(s));
  HCHECK(hipGetLastError());
  return HELM_OK;
}

// ---------------------------------------------------------------------------
// Krylov workspace layout (bytes, 256-aligned).
// ---------------------------------------------------------------------------
struct WsLayout {
  size_t Qi, X, W, V, Z, part, G, Gc, Hb, S, R, Rinv, Y, est, qn2, rn2, w2, hn2, nu, flag, act, ls, end;
};

// Storage of the outer Krylov basis V and work vector W: FP32 complex in
// mixed precision with block size 1 (every reduction over them stays FP64 and
// the residual is recomputed from FP64 Q and X at each restart), FP64 complex
// otherwise.
static Prec basis_prec(const helm_ctx* c, int pb) { return c->precision == HELM_MIXED && pb == 1 ? P32 : P64; }

static WsLayout ws_layout(const helm_ctx* c, int P, int m, int pb) {
  const int64_t N = c->lv[0].npts;
  const size_t blk = 16 * (size_t)N * P;
  const size_t vblk = psize(basis_prec(c, pb)) * (size_t)N * P;
  const size_t zblk = (c->precision == HELM_FP64 ? 16 : 8) * (size_t)N * P;
  const int ng = P / pb;
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  WsLayout w{};
  size_t o = 0;
  w.Qi = o; o += al(blk);
  w.X = o; o += al(blk);
  w.W = o; o += al(vblk);
  w.V = o; o += al(vblk) * (m + 1);
  w.Z = o; o += al(zblk) * m;
  w.part = o; o += al(16 * gram_part_elems(P));
  w.G = o; o += al(16 * (size_t)MAXPTR * P * pb);
  w.Gc = o; o += al(16 * (size_t)MAXPTR * P * pb);
  const size_t ldh = (size_t)(m + 1) * pb;
  w.Hb = o; o += al(16 * ldh * m * pb * ng);
  w.S = o; o += al(16 * (size_t)ng * pb * pb);
  w.R = o; o += al(16 * (size_t)ng * pb * pb);
  w.Rinv = o; o += al(16 * (size_t)ng * pb * pb);
  w.Y = o; o += al(16 * (size_t)m * P * pb);
  w.est = o; o += al(8 * (size_t)P);
  w.qn2 = o; o += al(8 * (size_t)P);
  w.rn2 = o; o += al(8 * (size_t)P);
  w.w2 = o; o += al(8 * (size_t)P);
  w.hn2 = o; o += al(8 * (size_t)P);
  w.nu = o; o += al(8 * (size_t)P * (m + 1));
  w.flag = o; o += al(4 * (size_t)ng);
  w.act = o; o += al(4 * (size_t)ng);
  w.ls = o; o += al(16 * (size_t)ng * (m + 1) * pb * (m + 1) * pb);
  w.end = o;
  return w;
}

// Block BiCGSTAB workspace: the FP64 blocks Q, X (and its copy at the last
// restart), R, the shadow Rt, the
// directions P (and its successor), V = H M P, S, T = H M S; the cycle
// outputs M P and M S in the cycle's precision; Gram and coefficient blocks.
struct BiWs {
  size_t Qi, X, Xr, R, Rt, Pp, Pn, V, S, T, Ph, Sh, part, G1, G2, G3, Al, Be, Cl, q2, r2, tn2, om, flag, act, end;
};

static BiWs bicg_layout(const helm_ctx* c, int P, int pb) {
  const int64_t N = c->lv[0].npts;
  const size_t blk = 16 * (size_t)N * P;
  const size_t zblk = (c->precision == HELM_FP64 ? 16 : 8) * (size_t)N * P;
  const int ng = (P + pb - 1) / pb;
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  BiWs w{};
  size_t o = 0;
  size_t* big[10] = {&w.Qi, &w.X, &w.Xr, &w.R, &w.Rt, &w.Pp, &w.Pn, &w.V, &w.S, &w.T};
  for (size_t* f : big) {
    *f = o;
    o += al(blk);
  }
  w.Ph = o; o += al(zblk);
  w.Sh = o; o += al(zblk);
  w.part = o; o += al(16 * gram_part_elems(P));
  const size_t gm = al(16 * (size_t)P * pb);
  w.G1 = o; o += gm;
  w.G2 = o; o += gm;
  w.G3 = o; o += gm;
  w.Al = o; o += gm;
  w.Be = o; o += gm;
  w.Cl = o; o += 3 * gm;
  w.q2 = o; o += al(8 * (size_t)P);
  w.r2 = o; o += al(8 * (size_t)P);
  w.tn2 = o; o += al(8 * (size_t)P);
  w.om = o; o += al(16 * (size_t)ng);
  w.flag = o; o += al(4 * (size_t)ng);
  w.act = o; o += al(4 * (size_t)ng);
  w.end = o;
  return w;
}

helm_status helm_workspace_size(helm_handle h, int32_t nrhs, int32_t restart, size_t* bytes) {
  if (!h || !bytes || nrhs < 1 || nrhs > 256 || restart < 1 || restart >= MAXPTR)
    return fail(HELM_ERR_INVALID_ARG, "bad workspace query");
  const int P = padP(nrhs);
  // enough for either method at any block size
  const size_t fg = std::max(ws_layout(h, P, restart, 1).end, ws_layout(h, P, restart, P).end);
  const size_t bi = std::max(bicg_layout(h, P, 1).end, bicg_layout(h, P, std::min(P, 32)).end);
  *bytes = std::max(fg, bi);
  return HELM_OK;
}

__global__ void k_hscatter(int pb, int j, int P, const c128* __restrict__ Gc, const c128* __restrict__ R,
                           c128* __restrict__ Hb, int ldh, int64_t hstride) {
  // block column j of Hbar for group g = blockIdx.x
  const int g = blockIdx.x;
  c128* H = Hb + (int64_t)g * hstride;
  const int rows = (j + 2) * pb;
  for (int e = threadIdx.x; e < rows * pb; e += blockDim.x) {
    const int row = e % rows, b = e / rows;
    const int i = row / pb, a = row % pb;
    c128 v;
    if (i <= j)
      v = Gc[((int64_t)i * P + g * pb + b) * pb + a];
    else
      v = R[((int64_t)g * pb + a) * pb + b];
    H[(int64_t)(j * pb + b) * ldh + row] = v;
  }
}


__global__ void k_set_active(int ng, int pb, double tol2, const double* __restrict__ rn2,
                             const double* __restrict__ qn2, int* __restrict__ act) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ng) return;
  int a = 0;
  for (int b = 0; b < pb; ++b) {
    const int c = g * pb + b;
    if (qn2[c] > 0.0 && rn2[c] > tol2 * qn2[c]) a = 1;
  }
  act[g] = a;
}

// Zero the update coefficients of inactive groups (their columns stay put).
__global__ void k_zero_inactive(int ng, int pb, int P, int k, const int* __restrict__ act, c128* __restrict__ C) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)k * P * pb) return;
  const int c = (int)((t / pb) % P);
  if (!act[c / pb]) C[t] = c128{0.0, 0.0};
}

// ---------------------------------------------------------------------------
// Block BiCGSTAB (El Guennouni, Jbilou and Sadok; the paper's W-BiCG of
// section 5.3) right-preconditioned by the multigrid cycle, per group of pb
// columns, all outer quantities in FP64:
//   R = Q - H X, Rt = R, P = R; per iteration
//   V = H M P, alpha = (Rt^H V)^-1 Rt^H R, S = R - V alpha,
//   T = H M S, omega = tr(T^H S) / tr(T^H T),
//   X += M P alpha + omega M S, R = S - omega T,
//   beta = -(Rt^H V)^-1 Rt^H T, P = R + (P - omega V) beta.
// When every active column's recursive residual meets tol (or a group's
// Rt^H V is singular), the FP64 true residual decides: stop, or restart from
// the current X. Converged groups get alpha = beta = omega = 0 and keep
// their columns. One host synchronisation per iteration.
// ---------------------------------------------------------------------------
static helm_status bicgstab_solve(helm_ctx* c, int nrhs, const void* Q, void* U, double tol, const helm_solve_opts& o,
                                  int pb, void* workspace, size_t ws_bytes, helm_solve_info* info, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int P = padP(nrhs);
  const int Pa = nrhs;
  const int ng = Pa / pb;
  const int64_t N = c->lv[0].npts;
  const Level& L0 = c->lv[0];
  const Prec pz = c->precision == HELM_FP64 ? P64 : P32;
  helm_status st;
  if ((st = ensure_fields(c, P)) != HELM_OK) return st;
  if ((st = autotune_fine(c, P, s)) != HELM_OK) return st;
  set_fine_tile(c->tile);
  const int64_t fallbacks0 = c->fallbacks;
  const int graph = (c->prof || c->cap) ? 0 : o.graph;
  const BiWs w = bicg_layout(c, P, pb);
  char* base = static_cast<char*>(workspace);
  if (!base) {
    if (c->wsbytes < w.end) {
      clear_graphs(c);
      hipFree(c->ws);
      c->ws = nullptr;
      c->wsbytes = 0;
      HCHECK(dmalloc(&c->ws, w.end));
      c->wsbytes = w.end;
    }
    base = static_cast<char*>(c->ws);
  } else if (ws_bytes < w.end) {
    return fail(HELM_ERR_INVALID_ARG, "workspace too small (%zu < %zu)", ws_bytes, w.end);
  }
  if (c->hbufn < (size_t)4 * P) {
    if (c->hbuf) hipHostFree(c->hbuf);
    HCHECK(hipHostMalloc(&c->hbuf, sizeof(double) * 4 * P));
    c->hbufn = 4 * P;
  }
  double* hq = c->hbuf;
  double* hr = c->hbuf + P;
  int* hflag = reinterpret_cast<int*>(c->hbuf + 2 * P);
  c128* Qi = (c128*)(base + w.Qi);
  c128* X = (c128*)(base + w.X);
  c128* Xr = (c128*)(base + w.Xr);
  c128* R = (c128*)(base + w.R);
  c128* Rt = (c128*)(base + w.Rt);
  c128* Pd = (c128*)(base + w.Pp);
  c128* Pn = (c128*)(base + w.Pn);
  c128* V = (c128*)(base + w.V);
  c128* S = (c128*)(base + w.S);
  c128* T = (c128*)(base + w.T);
  void* Ph = base + w.Ph;
  void* Sh = base + w.Sh;
  c128* part = (c128*)(base + w.part);
  c128* G1 = (c128*)(base + w.G1);
  c128* G2 = (c128*)(base + w.G2);
  c128* G3 = (c128*)(base + w.G3);
  c128* Al = (c128*)(base + w.Al);
  c128* Be = (c128*)(base + w.Be);
  c128* Cl = (c128*)(base + w.Cl);
  double* dq = (double*)(base + w.q2);
  double* dr = (double*)(base + w.r2);
  double* dtn = (double*)(base + w.tn2);
  c128* dom = (c128*)(base + w.om);
  int* dflag = (int*)(base + w.flag);
  int* dact = (int*)(base + w.act);
  const size_t blk = 16 * (size_t)N * P;
  const Geo g0 = L0.geo(P);
  const double tol2 = tol * tol;
  const Level& Lz = c->lv[0];

  hipEvent_t e0, e1;
  HCHECK(hipEventCreate(&e0));
  HCHECK(hipEventCreate(&e1));
  auto cleanup = [&]() {
    hipEventDestroy(e0);
    hipEventDestroy(e1);
  };
  HCHECK(hipEventRecord(e0, s));
  launch_to_internal(P64, N, nrhs, P, Q, Qi, s);
  if (o.warm_start)
    launch_to_internal(P64, N, nrhs, P, U, X, s);
  else
    HCHECK(hipMemsetAsync(X, 0, blk, s));
  if (o.op == HELM_OP_HH) {
    // H^H U = Q is conj(H) U = Q: solve H conj(U) = conj(Q) (H = H^T)
    launch_conj((int64_t)N * P, Qi, s);
    if (o.warm_start) launch_conj((int64_t)N * P, X, s);
  }
  { Prof pr_(c, HELM_K_GRAM, s); launch_colnorm2(P64, N, P, Pa, Qi, part, G1, dq, s); }
  HCHECK(hipMemcpyAsync(hq, dq, 8 * Pa, hipMemcpyDeviceToHost, s));
  HCHECK(hipStreamSynchronize(s));
  for (int cidx = 0; cidx < Pa; ++cidx)
    if (!std::isfinite(hq[cidx])) {
      cleanup();
      return fail(HELM_ERR_NONFINITE, "non-finite right-hand side column %d", cidx);
    }
  // the cycle M applied to a c128 block: FP64 directly, mixed through the
  // FP32 input field of the finest level
  auto precond = [&](const c128* in, void* out) -> helm_status {
    if (pz == P64) return run_cycle(c, P, in, out, Lz.U1, graph, s);
    launch_convert(P64, P32, N * P, in, Lz.F, s);
    return run_cycle(c, P, Lz.F, out, Lz.U1, graph, s);
  };
  auto apply_H = [&](const void* in, c128* out) {
    Prof pr(c, HELM_K_OUTER_APPLY, s);
    launch_fine(0, pz, P64, P64, P64, c->dim, g0, in, nullptr, out, L0.dH, nullptr, L0.ih, s);
  };
  int cycles = 0, restarts = 0;
  bool converged = false;
  std::vector<double> relres(Pa, 0.0);
  for (;;) {
    // true FP64 residual R = Q - H X and the stopping test
    launch_fine(1, P64, P64, P64, P64, c->dim, g0, X, Qi, R, L0.dH, nullptr, L0.ih, s);
    { Prof pr_(c, HELM_K_GRAM, s); launch_colnorm2(P64, N, P, Pa, R, part, G1, dr, s); }
    HCHECK(hipMemcpyAsync(hr, dr, 8 * Pa, hipMemcpyDeviceToHost, s));
    HCHECK(hipStreamSynchronize(s));
    HCHECK(hipGetLastError());
    bool all = true;
    for (int cidx = 0; cidx < Pa; ++cidx) {
      relres[cidx] = hq[cidx] > 0 ? std::sqrt(hr[cidx] / hq[cidx]) : 0.0;
      if (!std::isfinite(relres[cidx])) {
        cleanup();
        return fail(HELM_ERR_NONFINITE, "non-finite residual in column %d", cidx);
      }
      if (relres[cidx] > tol) all = false;
    }
    if (all) {
      converged = true;
      break;
    }
    if (cycles >= o.max_cycles) break;
    restarts += cycles > 0;
    hipLaunchKernelGGL(k_set_active, dim3((ng + 255) / 256), dim3(256), 0, s, ng, pb, tol2, dr, dq, dact);
    HCHECK(hipMemcpyAsync(Rt, R, blk, hipMemcpyDeviceToDevice, s));
    HCHECK(hipMemcpyAsync(Pd, R, blk, hipMemcpyDeviceToDevice, s));
    HCHECK(hipMemcpyAsync(Xr, X, blk, hipMemcpyDeviceToDevice, s));
    std::vector<double> r2start(hr, hr + Pa);
    bool diverged = false;
    PtrList rt{};
    rt.p[0] = Rt;
    bool stalled = true;  // no iteration completed since this restart
    while (cycles < o.max_cycles) {
      // V = H M P, alpha = (Rt^H V)^-1 Rt^H R
      if ((st = precond(Pd, Ph)) != HELM_OK) {
        cleanup();
        return st;
      }
      ++cycles;
      apply_H(Ph, V);
      {
        Prof pr_(c, HELM_K_GRAM, s);
        launch_gram(P64, N, P, Pa, pb, 1, rt, V, part, G1, s);
        launch_gram(P64, N, P, Pa, pb, 1, rt, R, part, G2, s);
      }
      launch_bicg_solve(ng, pb, 1.0, G1, G2, Al, dact, dflag, s);
      // S = R - V alpha
      launch_bicg_coefs(0, Pa, pb, Al, dom, Cl, s);
      {
        Prof pr_(c, HELM_K_UPDATE, s);
        PtrList vr{};
        vr.p[0] = V;
        vr.p[1] = R;
        launch_block_update(1, P64, P64, N, P, Pa, pb, 2, vr, Cl, S, s);
      }
      // T = H M S, omega = tr(T^H S) / tr(T^H T)
      if ((st = precond(S, Sh)) != HELM_OK) {
        cleanup();
        return st;
      }
      ++cycles;
      apply_H(Sh, T);
      {
        Prof pr_(c, HELM_K_GRAM, s);
        PtrList tl{};
        tl.p[0] = T;
        launch_gram(P64, N, P, Pa, pb, 1, tl, S, part, G3, s);
        launch_colnorm2(P64, N, P, Pa, T, part, G2, dtn, s);
      }
      launch_bicg_omega(ng, pb, G3, dtn, dact, dom, s);
      {
        Prof pr_(c, HELM_K_UPDATE, s);
        // X += M P alpha + omega M S
        launch_bicg_coefs(1, Pa, pb, Al, dom, Cl, s);
        PtrList ps{};
        ps.p[0] = Ph;
        ps.p[1] = Sh;
        launch_block_update(2, pz, P64, N, P, Pa, pb, 2, ps, Cl, X, s);
        // R = S - omega T
        launch_bicg_coefs(2, Pa, pb, nullptr, dom, Cl, s);
        PtrList st2{};
        st2.p[0] = S;
        st2.p[1] = T;
        launch_block_update(1, P64, P64, N, P, Pa, pb, 2, st2, Cl, R, s);
      }
      { Prof pr_(c, HELM_K_GRAM, s); launch_colnorm2(P64, N, P, Pa, R, part, G2, dr, s); }
      HCHECK(hipMemcpyAsync(hr, dr, 8 * Pa, hipMemcpyDeviceToHost, s));
      HCHECK(hipMemcpyAsync(hflag, dflag, 4 * ng, hipMemcpyDeviceToHost, s));
      HCHECK(hipStreamSynchronize(s));
      HCHECK(hipGetLastError());
      bool brk = false;
      for (int gg = 0; gg < ng; ++gg) brk = brk || hflag[gg];
      if (brk) break;  // singular Rt^H V: this step did nothing for that group; restart
      // divergence (a non-finite or exploding recursive residual, e.g. with
      // a cycle that is not linear enough): back to the restart's iterate
      for (int cidx = 0; cidx < Pa; ++cidx)
        if (!std::isfinite(hr[cidx]) || hr[cidx] > 1e16 * std::max(r2start[cidx], 1e-300)) diverged = true;
      if (diverged) break;
      stalled = false;
      bool conv = true;
      for (int cidx = 0; cidx < Pa; ++cidx)
        if (hq[cidx] > 0 && hr[cidx] > tol2 * hq[cidx]) conv = false;
      if (conv) break;
      // beta = -(Rt^H V)^-1 Rt^H T, P = R + (P - omega V) beta
      { Prof pr_(c, HELM_K_GRAM, s); launch_gram(P64, N, P, Pa, pb, 1, rt, T, part, G2, s); }
      launch_bicg_solve(ng, pb, -1.0, G1, G2, Be, dact, dflag, s);
      launch_bicg_coefs(3, Pa, pb, Be, dom, Cl, s);
      {
        Prof pr_(c, HELM_K_UPDATE, s);
        PtrList rpv{};
        rpv.p[0] = R;
        rpv.p[1] = Pd;
        rpv.p[2] = V;
        launch_block_update(1, P64, P64, N, P, Pa, pb, 3, rpv, Cl, Pn, s);
      }
      std::swap(Pd, Pn);
    }
    if (diverged) {
      HCHECK(hipMemcpyAsync(X, Xr, blk, hipMemcpyDeviceToDevice, s));
      if (o.op == HELM_OP_HH) launch_conj((int64_t)N * P, X, s);
      launch_to_abi(P64, N, nrhs, P, X, U, s);
      HCHECK(hipStreamSynchronize(s));
      cleanup();
      if (info) {
        info->cycles = cycles;
        info->restarts = restarts;
        info->converged_all = 0;
        info->fallback_used = (int32_t)(c->fallbacks - fallbacks0);
        info->t_solve_ms = 0.0;
        info->rate_switch = -1;
        for (int cidx = 0; cidx < nrhs; ++cidx) {
          if (info->relres) info->relres[cidx] = relres[cidx];
          if (info->converged) info->converged[cidx] = relres[cidx] <= tol;
        }
      }
      return fail(HELM_ERR_BREAKDOWN,
                  "block BiCGSTAB diverged after %d cycles (U holds the iterate of the last restart); BiCGSTAB "
                  "needs a linear cycle: use FP64 or FGMRES", cycles);
    }
    if (stalled) {
      // a breakdown in the first step after a (re)start cannot be cured by
      // restarting again (the flags were read with that step's residuals)
      bool any = false;
      for (int gg = 0; gg < ng; ++gg) any = any || hflag[gg];
      if (any) {
        cleanup();
        return fail(HELM_ERR_BREAKDOWN,
                    "block BiCGSTAB breakdown (singular shadow product) in a fresh start; dependent right-hand "
                    "sides in a group? use block_size 1");
      }
    }
  }
  if (o.op == HELM_OP_HH) launch_conj((int64_t)N * P, X, s);
  launch_to_abi(P64, N, nrhs, P, X, U, s);
  HCHECK(hipEventRecord(e1, s));
  HCHECK(hipEventSynchronize(e1));
  float ms = 0.f;
  hipEventElapsedTime(&ms, e0, e1);
  cleanup();
  HCHECK(hipGetLastError());
  if (info) {
    info->cycles = cycles;
    info->restarts = restarts;
    info->converged_all = converged ? 1 : 0;
    info->fallback_used = (int32_t)(c->fallbacks - fallbacks0);
    info->t_solve_ms = ms;
    info->rate_switch = -1;
    for (int cidx = 0; cidx < nrhs; ++cidx) {
      if (info->relres) info->relres[cidx] = relres[cidx];
      if (info->converged) info->converged[cidx] = relres[cidx] <= tol;
    }
  }
  if (!converged) return fail(HELM_ERR_NOT_CONVERGED, "not converged after %d cycles", cycles);
  return HELM_OK;
}

helm_status helm_solve_block(helm_handle h, int32_t nrhs, const void* Q, void* U, double tol,
                             const helm_solve_opts* opts, void* workspace, size_t ws_bytes, helm_solve_info* info,
                             void* stream) {
  helm_status st = check_block(h, nrhs, Q, U);
  if (st != HELM_OK) return st;
  if (!(tol > 0) || !std::isfinite(tol)) return fail(HELM_ERR_INVALID_ARG, "tol must be > 0");
  helm_solve_opts o{5, 1000, 0, 0, 2, 0, 0.0, 0, 0};
  if (opts) o = *opts;
  if (!(o.learned_rate >= 0.0 && o.learned_rate < 1.0))
    return fail(HELM_ERR_INVALID_ARG, "learned_rate must be in [0, 1)");
  const int m = o.restart;
  if (m < 1 || m >= MAXPTR) return fail(HELM_ERR_INVALID_ARG, "restart must be 1..%d", MAXPTR - 1);
  const int pb = o.block_size <= 0 ? nrhs : o.block_size;
  if (pb < 1 || nrhs % pb != 0 || pb > 64) return fail(HELM_ERR_INVALID_ARG, "block_size must divide nrhs and be <= 64");
  if (o.max_cycles < 1) return fail(HELM_ERR_INVALID_ARG, "max_cycles must be >= 1");
  if (o.reorth < 0 || o.reorth > 2) return fail(HELM_ERR_INVALID_ARG, "reorth must be 0, 1 or 2");
  if (o.graph < 0 || o.graph > 2) return fail(HELM_ERR_INVALID_ARG, "graph must be 0, 1 or 2");
  if (o.method != HELM_METHOD_FGMRES && o.method != HELM_METHOD_BICGSTAB)
    return fail(HELM_ERR_INVALID_ARG, "method must be HELM_METHOD_FGMRES or HELM_METHOD_BICGSTAB");
  if (o.op < HELM_OP_H || o.op > HELM_OP_HH) return fail(HELM_ERR_INVALID_ARG, "op must be HELM_OP_H, _HT or _HH");
  if (o.method == HELM_METHOD_BICGSTAB) return bicgstab_solve(h, nrhs, Q, U, tol, o, pb, workspace, ws_bytes, info, stream);
  hipStream_t s = static_cast<hipStream_t>(stream);
  helm_ctx* c = h;
  const int P = padP(nrhs);
  const int Pa = nrhs;  // active (real) columns
  const int ng = Pa / pb;
  const int64_t N = c->lv[0].npts;
  const Level& L0 = c->lv[0];
  const Prec pz = c->precision == HELM_FP64 ? P64 : P32;
  if ((st = ensure_fields(c, P)) != HELM_OK) return st;
  if ((st = autotune_fine(c, P, s)) != HELM_OK) return st;
  set_fine_tile(c->tile);
  const int64_t fallbacks0 = c->fallbacks;
  // graphs and the persistent kernel need a cycle without host work: no
  // per-kernel timing, no pair capture
  int graph = (c->prof || c->cap) ? 0 : o.graph;
  // per-cycle rate check of the learned coarsest correction: the block's
  // factor between restarts against sqrt of the calibrated plain factor
  const bool rate_check = o.learned_rate > 0.0 && c->coarse == HELM_COARSE_LEARNED && c->net;
  c->rate_fallback = false;
  int rate_switch = -1, rate_cycles0 = 0;
  double rate_res0 = 0.0;
  const WsLayout w = ws_layout(c, P, m, pb);
  char* base = static_cast<char*>(workspace);
  if (!base) {
    if (c->wsbytes < w.end) {
      clear_graphs(c);
      hipFree(c->ws);
      c->ws = nullptr;
      c->wsbytes = 0;
      HCHECK(dmalloc(&c->ws, w.end));
      c->wsbytes = w.end;
    }
    base = static_cast<char*>(c->ws);
  } else if (ws_bytes < w.end) {
    return fail(HELM_ERR_INVALID_ARG, "workspace too small (%zu < %zu)", ws_bytes, w.end);
  }
  if (c->hbufn < (size_t)4 * P) {
    if (c->hbuf) hipHostFree(c->hbuf);
    HCHECK(hipHostMalloc(&c->hbuf, sizeof(double) * 4 * P));
    c->hbufn = 4 * P;
  }
  double* hq = c->hbuf;          // ||q||^2
  double* hr = c->hbuf + P;      // ||r||^2
  double* hest = c->hbuf + 2 * P;
  int* hflag = reinterpret_cast<int*>(c->hbuf + 3 * P);
  const size_t blk = 16 * (size_t)N * P;
  const Prec pv = basis_prec(c, pb);
  c128* Qi = (c128*)(base + w.Qi);
  c128* X = (c128*)(base + w.X);
  void* W = base + w.W;
  std::vector<void*> V(m + 1);
  std::vector<void*> Z(m);
  const size_t vstride = (psize(pv) * (size_t)N * P + 255) / 256 * 256;
  const size_t zstride = ((pz == P64 ? 16 : 8) * (size_t)N * P + 255) / 256 * 256;
  for (int j = 0; j <= m; ++j) V[j] = base + w.V + j * vstride;
  for (int j = 0; j < m; ++j) Z[j] = base + w.Z + j * zstride;
  c128* part = (c128*)(base + w.part);
  c128* G = (c128*)(base + w.G);
  c128* Gc = (c128*)(base + w.Gc);
  c128* Hb = (c128*)(base + w.Hb);
  c128* S = (c128*)(base + w.S);
  c128* Rm = (c128*)(base + w.R);
  c128* Rinv = (c128*)(base + w.Rinv);
  c128* Yc = (c128*)(base + w.Y);
  double* dest = (double*)(base + w.est);
  double* dq = (double*)(base + w.qn2);
  double* dr = (double*)(base + w.rn2);
  double* dw2 = (double*)(base + w.w2);
  double* dhn2 = (double*)(base + w.hn2);
  double* dnu = (double*)(base + w.nu);
  int* dflag = (int*)(base + w.flag);
  int* dact = (int*)(base + w.act);
  c128* lsw = (c128*)(base + w.ls);
  const int ldh = (m + 1) * pb;
  const int64_t hstride = (int64_t)ldh * m * pb;
  const Geo g0 = L0.geo(P);
  // CholQR deflation: a column whose part independent of the columns
  // before it has a squared norm at most 1e-12 of its own (1e-6 in norm),
  // or 1e-26 of the group's largest, is dropped from the basis
  const double chol_tol = 1e-26, chol_rtol = 1e-12;

  hipEvent_t e0, e1;
  HCHECK(hipEventCreate(&e0));
  HCHECK(hipEventCreate(&e1));
  HCHECK(hipEventRecord(e0, s));
  launch_to_internal(P64, N, nrhs, P, Q, Qi, s);
  if (o.warm_start)
    launch_to_internal(P64, N, nrhs, P, U, X, s);
  else
    hipMemsetAsync(X, 0, blk, s);
  if (o.op == HELM_OP_HH) {
    // H^H U = Q is conj(H) U = Q: solve H conj(U) = conj(Q) (H = H^T)
    launch_conj((int64_t)N * P, Qi, s);
    if (o.warm_start) launch_conj((int64_t)N * P, X, s);
  }
  { Prof pr_(c, HELM_K_GRAM, s); launch_colnorm2(P64, N, P, Pa, Qi, part, G, dq, s); }
  HCHECK(hipMemcpyAsync(hq, dq, 8 * Pa, hipMemcpyDeviceToHost, s));
  HCHECK(hipStreamSynchronize(s));
  for (int cidx = 0; cidx < Pa; ++cidx)
    if (!std::isfinite(hq[cidx])) {
      hipEventDestroy(e0);
      hipEventDestroy(e1);
      return fail(HELM_ERR_NONFINITE, "non-finite right-hand side column %d", cidx);
    }
  int cycles = 0, restarts = 0;
  bool converged = false, breakdown = false;
  std::vector<double> relres(Pa, 0.0);
  std::vector<int> hact(ng, 1);
  const double tol2 = tol * tol;
  // W = Q R by CholQR (first pass into R, Q into Vb, W is consumed); where a
  // group dropped a column or lost orthogonality, a second pass
  // Q1 = Q2 R2 restores it and R becomes R2 R (R2 kept in the second
  // Gram slot of G).
  auto cholqr = [&](void*& Vb, c128* Rout) -> helm_status {
    PtrList wl{};
    wl.p[0] = W;
    { Prof pr_(c, HELM_K_GRAM, s); launch_gram(P64, N, P, Pa, pb, 1, wl, W, part, G, s); }
    launch_cholqr_small(ng, pb, G, Rout, Rinv, dflag, chol_tol, chol_rtol, s);
    hipLaunchKernelGGL(k_zero_inactive, dim3((P * pb + 255) / 256), dim3(256), 0, s, ng, pb, Pa, 1, dact, Rinv);
    { Prof pr_(c, HELM_K_UPDATE, s); launch_block_update(1, P64, P64, N, P, Pa, pb, 1, wl, Rinv, Vb, s); }
    HCHECK(hipMemcpyAsync(hflag, dflag, 4 * ng, hipMemcpyDeviceToHost, s));
    HCHECK(hipStreamSynchronize(s));
    bool ill = false;
    for (int gg = 0; gg < ng; ++gg) ill = ill || (hact[gg] && hflag[gg]);
    if (!ill) return HELM_OK;
    c128* R2 = G + (size_t)P * pb;
    PtrList ql{};
    ql.p[0] = Vb;
    { Prof pr_(c, HELM_K_GRAM, s); launch_gram(P64, N, P, Pa, pb, 1, ql, Vb, part, G, s); }
    launch_cholqr_small(ng, pb, G, R2, Rinv, dflag, chol_tol, chol_rtol, s);
    hipLaunchKernelGGL(k_zero_inactive, dim3((P * pb + 255) / 256), dim3(256), 0, s, ng, pb, Pa, 1, dact, Rinv);
    { Prof pr_(c, HELM_K_UPDATE, s); launch_block_update(1, P64, P64, N, P, Pa, pb, 1, ql, Rinv, W, s); }
    std::swap(Vb, W);
    launch_rmul_small(ng, pb, R2, Rout, s);
    return HELM_OK;
  };
  for (;;) {
    // true FP64 residual R = Q - H X into V0
    launch_fine(1, P64, P64, pv, P64, c->dim, g0, X, Qi, V[0], L0.dH, nullptr, L0.ih, s);
    { Prof pr_(c, HELM_K_GRAM, s); launch_colnorm2(pv, N, P, Pa, V[0], part, G, dr, s); }
    HCHECK(hipMemcpyAsync(hr, dr, 8 * Pa, hipMemcpyDeviceToHost, s));
    HCHECK(hipStreamSynchronize(s));
    HCHECK(hipGetLastError());
    bool all = true;
    for (int cidx = 0; cidx < Pa; ++cidx) {
      relres[cidx] = hq[cidx] > 0 ? std::sqrt(hr[cidx] / hq[cidx]) : 0.0;
      if (!std::isfinite(relres[cidx])) {
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        return fail(HELM_ERR_NONFINITE, "non-finite residual in column %d", cidx);
      }
      if (relres[cidx] > tol) all = false;
    }
    if (all) {
      converged = true;
      break;
    }
    if (rate_check && !c->rate_fallback) {
      double worst = 0.0;
      for (int cidx = 0; cidx < Pa; ++cidx) worst = std::max(worst, relres[cidx]);
      if (cycles > rate_cycles0 && rate_res0 > 0.0) {
        const double rho = std::pow(worst / rate_res0, 1.0 / (cycles - rate_cycles0));
        if (rho > std::sqrt(o.learned_rate)) {
          // the rest of the solve runs the GMRES fallback on the coarsest grid
          // (eagerly: captured graphs hold the network's path)
          c->rate_fallback = true;
          rate_switch = cycles;
          graph = 0;
        }
      }
      rate_res0 = worst;
      rate_cycles0 = cycles;
    }
    if (cycles >= o.max_cycles || breakdown) break;
    restarts += cycles > 0;
    hipLaunchKernelGGL(k_set_active, dim3((ng + 255) / 256), dim3(256), 0, s, ng, pb, tol2, dr, dq, dact);
    // V0 S = R: CholQR, or plain normalisation for block size 1
    {
      HCHECK(hipMemcpyAsync(hact.data(), dact, 4 * ng, hipMemcpyDeviceToHost, s));
      if (pb == 1) {
        // unnormalised basis: v~_0 = r with nu_0 = ||r|| (no scaling pass)
        launch_lazy_start(Pa, dr, dnu, S, dflag, s);
      } else {
        // R = V_0 S; dependent residual columns (duplicate or combined
        // sources) leave zero columns in V_0
        std::swap(V[0], W);
        st = cholqr(V[0], S);
        if (st != HELM_OK) {
          hipEventDestroy(e0);
          hipEventDestroy(e1);
          return st;
        }
      }
      HCHECK(hipMemsetAsync(Hb, 0, 16 * (size_t)hstride * ng, s));
      HCHECK(hipStreamSynchronize(s));
    }
    int jlast = -1;
    for (int j = 0; j < m; ++j) {
      // Z_j = cycle(V_j)
      const Level& Lz = c->lv[0];
      if (pz == P64 || pv == P32) {
        st = run_cycle(c, P, V[j], Z[j], Lz.U1, graph, s);
      } else {
        launch_convert(P64, P32, N * P, V[j], Lz.F, s);
        st = run_cycle(c, P, Lz.F, Z[j], Lz.U1, graph, s);
      }
      if (st != HELM_OK) {
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        return st;
      }
      ++cycles;
      // W = H Z_j (FP64)
      {
        Prof pr(c, HELM_K_OUTER_APPLY, s);
        launch_fine(0, pz, pv == P32 ? P32 : P64, pv, P64, c->dim, g0, Z[j], nullptr, W, L0.dH, nullptr, L0.ih, s);
      }
      // block classical Gram-Schmidt against V_0..V_j, then W = V_{j+1} R
      PtrList vl{};
      for (int i = 0; i <= j; ++i) vl.p[i] = V[i];
      if (pb == 1) {
        // One pass gives v~_i^H W~ and ||W~||^2, the update returns ||W~'||^2;
        // a second pass runs when asked (reorth 1) or where the norm fell
        // below half (reorth 2, the "twice is enough" test). The new vector
        // is kept unnormalised (nu_{j+1} = its norm), so W~' becomes v~_{j+1}.
        PtrList vw = vl;
        vw.p[j + 1] = W;
        { Prof pr_(c, HELM_K_GRAM, s); launch_gram(pv, N, P, Pa, 1, j + 2, vw, W, part, G, s); }
        launch_diag_real(Pa, G + (size_t)(j + 1) * Pa, dw2, s);
        launch_lazy_coef(Pa, j, G, dnu, Gc, Hb, ldh, hstride, 0, s);
        { Prof pr_(c, HELM_K_UPDATE, s); launch_update_norm(pv, N, P, Pa, j + 1, vl, Gc, W, part, G + (size_t)(j + 2) * Pa, dhn2, s); }
        bool again = o.reorth == 1;
        if (o.reorth == 2) {
          std::vector<double> a(Pa), b(Pa);
          HCHECK(hipMemcpyAsync(a.data(), dw2, 8 * Pa, hipMemcpyDeviceToHost, s));
          HCHECK(hipMemcpyAsync(b.data(), dhn2, 8 * Pa, hipMemcpyDeviceToHost, s));
          HCHECK(hipStreamSynchronize(s));
          for (int cidx = 0; cidx < Pa; ++cidx)
            if (hact[cidx] && b[cidx] < 0.25 * a[cidx]) again = true;
        }
        if (again) {
          { Prof pr_(c, HELM_K_GRAM, s); launch_gram(pv, N, P, Pa, 1, j + 1, vl, W, part, G, s); }
          launch_lazy_coef(Pa, j, G, dnu, Gc, Hb, ldh, hstride, 1, s);
          { Prof pr_(c, HELM_K_UPDATE, s); launch_update_norm(pv, N, P, Pa, j + 1, vl, Gc, W, part, G + (size_t)(j + 2) * Pa, dhn2, s); }
        }
        launch_lazy_next(Pa, j, dhn2, dw2, 1e-28, dnu, Hb, ldh, hstride, dflag, s);
        std::swap(V[j + 1], W);
      } else {
        { Prof pr_(c, HELM_K_GRAM, s); launch_gram(P64, N, P, Pa, pb, j + 1, vl, W, part, Gc, s); }
        { Prof pr_(c, HELM_K_UPDATE, s); launch_block_update(0, P64, P64, N, P, Pa, pb, j + 1, vl, Gc, W, s); }
        if (o.reorth) {
          { Prof pr_(c, HELM_K_GRAM, s); launch_gram(P64, N, P, Pa, pb, j + 1, vl, W, part, G, s); }
          { Prof pr_(c, HELM_K_UPDATE, s); launch_block_update(0, P64, P64, N, P, Pa, pb, j + 1, vl, G, W, s); }
          const int64_t ne = (int64_t)(j + 1) * Pa * pb;
          hipLaunchKernelGGL(helm::k_add_c128, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, ne, G, Gc);
        }
        st = cholqr(V[j + 1], Rm);  // W = V_{j+1} H_{j+1,j}
        if (st != HELM_OK) {
          hipEventDestroy(e0);
          hipEventDestroy(e1);
          return st;
        }
      }
      if (pb > 1) hipLaunchKernelGGL(k_hscatter, dim3(ng), dim3(256), 0, s, pb, j, Pa, Gc, Rm, Hb, ldh, hstride);
      launch_block_ls(ng, pb, j, Hb, ldh, hstride, S, Yc, 0, dest, lsw, dact, s);
      HCHECK(hipMemcpyAsync(hest, dest, 8 * Pa, hipMemcpyDeviceToHost, s));
      HCHECK(hipMemcpyAsync(hflag, dflag, 4 * ng, hipMemcpyDeviceToHost, s));
      HCHECK(hipStreamSynchronize(s));
      HCHECK(hipGetLastError());
      bool conv = true;
      for (int cidx = 0; cidx < Pa; ++cidx)
        if (hq[cidx] > 0 && hest[cidx] > tol * std::sqrt(hq[cidx])) conv = false;
      // block size 1: a vanishing new basis vector ends the cycle (the
      // Krylov space is invariant); larger blocks drop dependent columns
      bool brk = false;
      if (pb == 1)
        for (int gg = 0; gg < ng; ++gg) brk = brk || (hact[gg] && hflag[gg]);
      jlast = j;
      if (conv || brk || j == m - 1 || cycles >= o.max_cycles) break;
    }
    // X += sum_j Z_j Y_j (block size 1: the stored z~_j carry the factor nu_j)
    if (pb == 1) launch_lazy_y(Pa, jlast + 1, dnu, Yc, s);
    hipLaunchKernelGGL(k_zero_inactive, dim3((unsigned)(((jlast + 1) * P * pb + 255) / 256)), dim3(256), 0, s, ng,
                       pb, Pa, jlast + 1, dact, Yc);
    PtrList zl{};
    for (int i = 0; i <= jlast; ++i) zl.p[i] = Z[i];
    { Prof pr_(c, HELM_K_UPDATE, s); launch_block_update(2, pz, P64, N, P, Pa, pb, jlast + 1, zl, Yc, X, s); }
  }
  if (o.op == HELM_OP_HH) launch_conj((int64_t)N * P, X, s);
  launch_to_abi(P64, N, nrhs, P, X, U, s);
  HCHECK(hipEventRecord(e1, s));
  HCHECK(hipEventSynchronize(e1));
  float ms = 0.f;
  hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  HCHECK(hipGetLastError());
  if (info) {
    info->cycles = cycles;
    info->restarts = restarts;
    info->converged_all = converged ? 1 : 0;
    info->fallback_used = (int32_t)(c->fallbacks - fallbacks0);
    info->t_solve_ms = ms;
    info->rate_switch = rate_switch;
    for (int cidx = 0; cidx < nrhs; ++cidx) {
      if (info->relres) info->relres[cidx] = relres[cidx];
      if (info->converged) info->converged[cidx] = relres[cidx] <= tol;
    }
  }
  c->rate_fallback = false;
  if (!converged) return fail(HELM_ERR_NOT_CONVERGED, "not converged after %d cycles", cycles);
  return HELM_OK;
}

helm_status helm_residual(helm_handle h, int32_t nrhs, const void* Q, const void* U, double* relres, void* stream) {
  helm_status st = check_block(h, nrhs, Q, U);
  if (st != HELM_OK) return st;
  if (!relres) return fail(HELM_ERR_INVALID_ARG, "relres is null");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Level& L = h->lv[0];
  // partial sums of the one-pass residual kernel: a buffer of the largest
  // size (RESID_MAX_COLS columns), allocated on the first call and kept
  if (!h->resid_buf) {
    const size_t n = (size_t)RESID_MAX_COLS * (2 * RESID_MAX_CHUNKS + 1);
    HCHECK(dmalloc(&h->resid_buf, sizeof(double) * n));
  }
  launch_resid_norms(L.geo(1), nrhs, L.ih, L.dH, Q, U, h->resid_buf, s);
  HCHECK(hipGetLastError());
  HCHECK(hipMemcpyAsync(relres, h->resid_buf, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
  HCHECK(hipStreamSynchronize(s));
  return HELM_OK;
}

helm_status helm_fields_pack16(helm_handle h, int32_t nrhs, const void* U, void* U16, double* scales, void* stream) {
  helm_status st = check_block(h, nrhs, U, U16);
  if (st != HELM_OK) return st;
  if (!scales) return fail(HELM_ERR_INVALID_ARG, "scales is null");
  launch_pack16(h->lv[0].npts, nrhs, static_cast<const c128*>(U), scales, U16, static_cast<hipStream_t>(stream));
  HCHECK(hipGetLastError());
  return HELM_OK;
}

helm_status helm_fields_unpack16(helm_handle h, int32_t nrhs, const void* U16, const double* scales, void* U,
                                 void* stream) {
  helm_status st = check_block(h, nrhs, U16, U);
  if (st != HELM_OK) return st;
  if (!scales) return fail(HELM_ERR_INVALID_ARG, "scales is null");
  launch_unpack16(h->lv[0].npts, nrhs, U16, scales, static_cast<c128*>(U), static_cast<hipStream_t>(stream));
  HCHECK(hipGetLastError());
  return HELM_OK;
}

static helm_status check_fields(const void* U, const void* U16, const double* scales) {
  if ((U == nullptr) == (U16 == nullptr)) return fail(HELM_ERR_INVALID_ARG, "give the fields as U or as U16");
  if (U16 && !scales) return fail(HELM_ERR_INVALID_ARG, "16-bit fields need their scales");
  return HELM_OK;
}

helm_status helm_jvp(helm_handle h, int32_t nrhs, const void* U, const void* U16, const double* scales,
                     const double* dm, void* JV, double tol, const helm_solve_opts* opts, helm_solve_info* info,
                     void* stream) {
  helm_status st = check_block(h, nrhs, U ? U : U16, JV);
  if (st != HELM_OK) return st;
  if ((st = check_fields(U, U16, scales)) != HELM_OK) return st;
  if (!dm) return fail(HELM_ERR_INVALID_ARG, "dm is null");
  hipStream_t s = static_cast<hipStream_t>(stream);
  helm_solve_opts o{5, 1000, 0, 0, 2, 0, 0.0, 0, 0};
  if (opts) o = *opts;
  o.op = HELM_OP_H;
  o.warm_start = 0;
  // right-hand side omega^2 (1 - i gamma) u dm into JV, then H JV = JV (the
  // solve copies its right-hand side before it writes its solution)
  launch_jvp_rhs(h->lv[0].npts, nrhs, h->lv[0].dS, U, U16, scales, dm, static_cast<c128*>(JV), s);
  HCHECK(hipGetLastError());
  return helm_solve_block(h, nrhs, JV, JV, tol, &o, nullptr, 0, info, stream);
}

helm_status helm_jtvp(helm_handle h, int32_t nrhs, const void* U, const void* U16, const double* scales,
                      const void* W, double* g, double tol, const helm_solve_opts* opts, helm_solve_info* info,
                      void* stream) {
  helm_status st = check_block(h, nrhs, U ? U : U16, W);
  if (st != HELM_OK) return st;
  if ((st = check_fields(U, U16, scales)) != HELM_OK) return st;
  if (!g) return fail(HELM_ERR_INVALID_ARG, "g is null");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t N = h->lv[0].npts;
  const size_t need = 16 * (size_t)N * nrhs;
  if (h->sensbytes < need) {
    hipFree(h->sensbuf);
    h->sensbuf = nullptr;
    h->sensbytes = 0;
    HCHECK(dmalloc(&h->sensbuf, need));
    h->sensbytes = need;
  }
  helm_solve_opts o{5, 1000, 0, 0, 2, 0, 0.0, 0, 0};
  if (opts) o = *opts;
  o.op = HELM_OP_HH;
  o.warm_start = 0;
  c128* Y = static_cast<c128*>(h->sensbuf);
  st = helm_solve_block(h, nrhs, W, Y, tol, &o, nullptr, 0, info, stream);
  if (st != HELM_OK) return st;
  launch_jtvp_accum(N, nrhs, h->lv[0].dS, U, U16, scales, Y, g, s);
  HCHECK(hipGetLastError());
  HCHECK(hipStreamSynchronize(s));
  return HELM_OK;
}

helm_status helm_residual_noalloc(helm_handle h, int32_t nrhs, const void* Q, const void* U, double* relres,
                                  void* stream) {
  if (!h) return fail(HELM_ERR_INVALID_ARG, "null handle");
  if (nrhs < 1 || nrhs > RESID_MAX_COLS)
    return fail(HELM_ERR_INVALID_ARG, "nrhs must be 1..%d (the size of the static scratch)", RESID_MAX_COLS);
  if (!Q || !U) return fail(HELM_ERR_INVALID_ARG, "null device pointer");
  if (!relres) return fail(HELM_ERR_INVALID_ARG, "relres is null");
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* scr = nullptr;
  HCHECK(resid_static_scratch(&scr));
  const Level& L = h->lv[0];
  // every partial that k_resid_final reads is written by k_resid_part first,
  // so the array's contents from an earlier call need no clearing
  launch_resid_norms(L.geo(1), nrhs, L.ih, L.dH, Q, U, scr, s);
  HCHECK(hipGetLastError());
  HCHECK(hipMemcpyAsync(relres, scr, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
  HCHECK(hipStreamSynchronize(s));
  return HELM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Learned coarsest-grid correction: network objects.
// ---------------------------------------------------------------------------
struct helm_net_s {
  learned::Net* n = nullptr;
  hipStream_t s = nullptr;
  // handles whose coarsest solves feed this network's pool: detached when
  // either side is destroyed, so no handle keeps a pointer to a freed pool
  std::vector<helm_ctx*> attached;
};

static void cap_detach(helm_ctx* h) {
  if (!h || !h->capw) return;
  auto& a = h->capw->attached;
  a.erase(std::remove(a.begin(), a.end(), h), a.end());
  h->cap = nullptr;
  h->capw = nullptr;
}

static void cap_attach(helm_ctx* h, helm_net_s* n) {
  if (h->capw != n) {
    cap_detach(h);
    n->attached.push_back(h);
  }
  h->cap = n->n;
  h->capw = n;
}

int64_t helm_net_nparams(void) { return learned::nparams(); }

helm_status helm_net_create(int32_t D, int32_t max_batch, uint64_t seed, void* stream, helm_net* out) {
  if (!out) return fail(HELM_ERR_INVALID_ARG, "null output");
  *out = nullptr;
  helm_net_s* w = new helm_net_s();
  w->s = static_cast<hipStream_t>(stream);
  const helm_status st = learned::create(D, max_batch, seed, w->s, &w->n);
  if (st != HELM_OK) {
    delete w;
    return st;
  }
  *out = w;
  return HELM_OK;
}

void helm_net_destroy(helm_net n) {
  if (!n) return;
  while (!n->attached.empty()) cap_detach(n->attached.back());
  learned::destroy(n->n);
  delete n;
}

helm_status helm_net_set_params(helm_net n, const float* params) {
  if (!n || !params) return fail(HELM_ERR_INVALID_ARG, "null argument");
  return learned::set_params(n->n, params, n->s);
}

helm_status helm_net_get_params(helm_net n, float* params) {
  if (!n || !params) return fail(HELM_ERR_INVALID_ARG, "null argument");
  return learned::get_params(n->n, params, n->s);
}

helm_status helm_net_get_state(helm_net n, float* state, int64_t* step) {
  if (!n || !state || !step) return fail(HELM_ERR_INVALID_ARG, "null argument");
  return learned::get_state(n->n, state, step, n->s);
}

helm_status helm_net_set_state(helm_net n, const float* state, int64_t step) {
  if (!n || !state) return fail(HELM_ERR_INVALID_ARG, "null argument");
  return learned::set_state(n->n, state, step, n->s);
}

helm_status helm_net_save(helm_net n, void* blob, size_t* bytes) {
  if (!n || !bytes) return fail(HELM_ERR_INVALID_ARG, "null argument");
  if (!blob) {
    *bytes = learned::blob_bytes();
    return HELM_OK;
  }
  if (*bytes < learned::blob_bytes()) return fail(HELM_ERR_INVALID_ARG, "blob needs %zu bytes", learned::blob_bytes());
  *bytes = learned::blob_bytes();
  return learned::write_blob(n->n, blob, n->s);
}

helm_status helm_net_forward(helm_net n, int32_t B, const float* x, float* out, void* stream) {
  if (!n) return fail(HELM_ERR_INVALID_ARG, "null network");
  return learned::forward(n->n, B, x, out, static_cast<hipStream_t>(stream));
}

helm_status helm_net_loss_grad(helm_net n, int32_t B, const float* x, const float* target, const uint8_t* mask,
                               float* grad, double* loss, void* stream) {
  if (!n) return fail(HELM_ERR_INVALID_ARG, "null network");
  return learned::loss_grad(n->n, B, x, target, mask, grad, loss, static_cast<hipStream_t>(stream));
}

helm_status helm_net_train_step(helm_net n, int32_t B, const float* x, const float* target, const uint8_t* mask,
                               double lr, double* loss, void* stream) {
  if (!n) return fail(HELM_ERR_INVALID_ARG, "null network");
  return learned::train_step(n->n, B, x, target, mask, lr, loss, static_cast<hipStream_t>(stream));
}

helm_status helm_net_capture(helm_handle h, helm_net n, int32_t max_pairs) {
  if (!h || !n) return fail(HELM_ERR_INVALID_ARG, "null argument");
  if (max_pairs == 0) {
    if (h->capw == n) cap_detach(h);
    return HELM_OK;
  }
  if (h->dim != 3) return fail(HELM_ERR_UNSUPPORTED, "pairs are captured from 3D problems only");
  if (h->coarse != HELM_COARSE_LU && h->coarse != HELM_COARSE_GMRES)
    return fail(HELM_ERR_INVALID_ARG, "pairs need an LU or GMRES coarsest solve");
  if (max_pairs < 0) {
    // keep the pool: pairs of several problems with equal coarsest grids
    helm_status st = learned::capture_continue(n->n, coarse_view(h), n->s);
    if (st != HELM_OK) return st;
    cap_attach(h, n);
    return HELM_OK;
  }
  helm_status st = learned::bind(n->n, coarse_view(h), n->s);
  if (st != HELM_OK) return st;
  if ((st = learned::capture_begin(n->n, max_pairs)) != HELM_OK) return st;
  cap_attach(h, n);
  return HELM_OK;
}

int64_t helm_net_pairs(helm_net n) { return n ? learned::pairs(n->n) : 0; }

helm_status helm_net_pool_read(helm_net n, int64_t i, float* x, float* target, void* stream) {
  if (!n) return fail(HELM_ERR_INVALID_ARG, "null network");
  return learned::pool_read(n->n, i, x, target, static_cast<hipStream_t>(stream));
}

helm_status helm_net_train(helm_net n, int32_t steps, int32_t batch, double lr, uint64_t seed, double* hist,
                           void* stream) {
  if (!n) return fail(HELM_ERR_INVALID_ARG, "null network");
  return learned::train(n->n, steps, batch, lr, seed, hist, static_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------------------
// Independent instances solved concurrently: each handle works on a stream of
// its own, driven by one of a pool of host threads (every solve synchronises
// its own stream once per Arnoldi step, so a thread per active instance keeps
// the GPU fed with the other instances' kernels meanwhile).
// ---------------------------------------------------------------------------
// k hierarchies from k descriptors (e.g. one model at several frequencies,
// as frequency continuation needs), set up one after another on `stream`.
helm_status helm_setup_batch(int32_t k, const helm_setup_desc* descs, void* stream, helm_handle* out) {
  if (k < 1 || !descs || !out) return fail(HELM_ERR_INVALID_ARG, "bad batch set-up arguments");
  for (int i = 0; i < k; ++i) out[i] = nullptr;
  for (int i = 0; i < k; ++i) {
    const helm_status st = helm_setup(&descs[i], stream, &out[i]);
    if (st != HELM_OK) {
      const std::string msg = "instance " + std::to_string(i) + ": " + g_err;
      for (int j = 0; j < i; ++j) {
        helm_destroy(out[j]);
        out[j] = nullptr;
      }
      g_err = msg;
      return st;
    }
  }
  return HELM_OK;
}

helm_status helm_solve_batch(int32_t k, const helm_handle* hs, const int32_t* nrhs, const void* const* Q,
                             void* const* U, double tol, const helm_solve_opts* opts, helm_solve_info* infos,
                             int32_t* status, int32_t max_threads, void* stream) {
  if (k < 1 || !hs || !nrhs || !Q || !U) return fail(HELM_ERR_INVALID_ARG, "bad batch arguments");
  // cooperative launches on concurrent streams could each hold part of the
  // device while waiting for the rest of their grid
  if (opts && opts->graph == 2)
    return fail(HELM_ERR_INVALID_ARG, "the persistent cycle (graph 2) is not available in a concurrent batch");
  for (int i = 0; i < k; ++i) {
    if (!hs[i]) return fail(HELM_ERR_INVALID_ARG, "null handle at %d", i);
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail(HELM_ERR_INVALID_ARG, "handle %d appears twice (instances need their own)", i);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0;
  HCHECK(hipGetDevice(&dev));
  for (int i = 0; i < k; ++i)
    if (!hs[i]->bstream) HCHECK(hipStreamCreateWithFlags(&hs[i]->bstream, hipStreamNonBlocking));
  // inputs written on the caller's stream are visible to every instance
  hipEvent_t ready;
  HCHECK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  HCHECK(hipEventRecord(ready, s));
  for (int i = 0; i < k; ++i) HCHECK(hipStreamWaitEvent(hs[i]->bstream, ready, 0));
  std::vector<helm_status> st(k, HELM_OK);
  std::vector<std::string> msg(k);
  std::atomic<int> next{0};
  auto worker = [&]() {
    (void)hipSetDevice(dev);
    for (;;) {
      const int i = next.fetch_add(1);
      if (i >= k) break;
      st[i] = helm_solve_block(hs[i], nrhs[i], Q[i], U[i], tol, opts, nullptr, 0, infos ? &infos[i] : nullptr,
                               hs[i]->bstream);
      if (st[i] != HELM_OK) msg[i] = g_err;
    }
  };
  const int nt = std::max(1, std::min(k, max_threads > 0 ? max_threads : 16));
  std::vector<std::thread> pool;
  pool.reserve(nt);
  for (int t = 0; t < nt; ++t) pool.emplace_back(worker);
  for (auto& t : pool) t.join();
  (void)hipEventDestroy(ready);
  // the caller's stream continues after every instance
  for (int i = 0; i < k; ++i) {
    hipEvent_t done;
    HCHECK(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    HCHECK(hipEventRecord(done, hs[i]->bstream));
    HCHECK(hipStreamWaitEvent(s, done, 0));
    (void)hipEventDestroy(done);
  }
  helm_status first = HELM_OK;
  for (int i = 0; i < k; ++i) {
    if (status) status[i] = st[i];
    if (st[i] != HELM_OK && first == HELM_OK) {
      first = st[i];
      g_err = "instance " + std::to_string(i) + ": " + msg[i];
    }
  }
  return first;
}
