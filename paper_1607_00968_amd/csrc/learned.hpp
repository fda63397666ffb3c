// learned.hpp -- learned coarsest-grid correction (convolutional network).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/helm.h"

struct helm_ctx;

namespace helm {
namespace learned {
struct Net;
helm_status create(helm_ctx* c, const void* blob, size_t bytes, Net** out, hipStream_t s);
void destroy(Net* n);
void apply(Net* n, helm_ctx* c, int level, int P, const void* f, void* out, hipStream_t s);
int fallback_used(const Net* n);
}  // namespace learned
}  // namespace helm
