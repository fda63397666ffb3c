// learned.hpp -- learned coarsest-grid correction (convolutional network).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/helm.h"
#include "kernels.hpp"

namespace helm {

// Records an error message for helm_last_error and returns st.
helm_status fail(helm_status st, const char* fmt, ...);

namespace learned {

struct Net;

// The coarsest grid as the network sees it.
struct Coarse {
  int nu[3];       // unknowns per axis
  double H2;       // squared mesh width of the coarsest grid
  Prec p;          // storage of the coarsest fields (P64 or P32)
  const c128* st;  // [N][27] Galerkin stencil, centre tap 13
};

int64_t nparams();
// Edge of the cubic volume the coarsest grid is embedded in (multiple of 4).
int edge_for(const Coarse& g);

// A network on D^3 volumes that processes up to max_batch samples per pass;
// parameters drawn with He scaling from `seed`.
helm_status create(int D, int max_batch, uint64_t seed, hipStream_t s, Net** out);
void destroy(Net* n);
helm_status set_params(Net* n, const float* host, hipStream_t s);
helm_status get_params(Net* n, float* host, hipStream_t s);
helm_status get_state(Net* n, float* host, int64_t* step, hipStream_t s);
helm_status set_state(Net* n, const float* host, int64_t step, hipStream_t s);
// Weights blob: "HNET", uint32 version 1, int64 nparams, float params[].
size_t blob_bytes();
helm_status write_blob(Net* n, void* blob, hipStream_t s);
helm_status read_blob(const void* blob, size_t bytes, float* params);

// Device FP32 in/out: x [B][D^3][4] -> out [B][D^3][2], B <= max_batch.
helm_status forward(Net* n, int B, const float* x, float* out, hipStream_t s);
// Loss (mean relative squared error on mask) and its gradient [nparams]
// (device) at x, target [B][D^3][2], mask [D^3] (device).
helm_status loss_grad(Net* n, int B, const float* x, const float* target, const uint8_t* mask, float* grad,
                      double* loss, hipStream_t s);

// Binds the network to a coarsest grid (input channels, scales, mask).
helm_status bind(Net* n, const Coarse& g, hipStream_t s);
// out = network correction for the P columns of f ([Nc][P] fields of the
// bound precision). Returns false when an output is not finite or beyond 1e4 in
// the normalised units (host sync).
bool apply(Net* n, int P, const void* f, void* out, hipStream_t s);
// The same without the host check (for graph capture): scratch for P columns
// must exist (prepare), and the non-finite count stays on the device until
// bad_count reads it (synchronises s; -1 on a device error).
helm_status prepare(Net* n, int P);
void apply_async(Net* n, int P, const void* f, void* out, hipStream_t s);
int bad_count(Net* n, hipStream_t s);
// Changes whenever prepare/apply move the per-column scratch (captured graphs
// that reference it are then stale).
uint64_t scratch_gen(const Net* n);

// Training pairs (f, e = exact coarsest solution) of the bound grid, kept by
// reservoir sampling in a pool of max_pairs volumes.
helm_status capture_begin(Net* n, int max_pairs);
// Binds to another coarsest grid of the same dimensions and keeps the pool
// (pairs from several problems in one pool).
helm_status capture_continue(Net* n, const Coarse& g, hipStream_t s);
void capture(Net* n, int P, const void* f, const void* e, hipStream_t s);
int64_t pairs(const Net* n);
// Copy pool entry i: x [D^3][4] and target [D^3][2], device FP32.
helm_status pool_read(Net* n, int64_t i, float* x, float* t, hipStream_t s);
// Adam on random minibatches of the pool; hist[steps] gets the loss per step.
helm_status train(Net* n, int steps, int batch, double lr, uint64_t seed, double* hist, hipStream_t s);
// One Adam step on a caller-supplied minibatch (no sampling, no phase turn).
helm_status train_step(Net* n, int B, const float* x, const float* target, const uint8_t* mask, double lr,
                       double* loss, hipStream_t s);

}  // namespace learned
}  // namespace helm
