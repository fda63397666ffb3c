// learned.hip -- learned coarsest-grid correction (placeholder until the
// network kernels are in).
#include "learned.hpp"
#include "kernels.hpp"

namespace helm {
namespace learned {
struct Net {
  int fallback = 0;
};
helm_status create(helm_ctx*, const void*, size_t, Net** out, hipStream_t) {
  *out = nullptr;
  return HELM_ERR_UNSUPPORTED;
}
void destroy(Net* n) { delete n; }
void apply(Net*, helm_ctx*, int, int, const void*, void*, hipStream_t) {}
int fallback_used(const Net* n) { return n ? n->fallback : 0; }
}  // namespace learned
}  // namespace helm
