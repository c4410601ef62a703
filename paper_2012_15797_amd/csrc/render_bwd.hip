// Adjoint of the forward render (placeholder until the adjoint kernels land).
#include "gfc_internal.hpp"

extern "C" {
size_t gfc_backward_workspace_bytes(int64_t n) { return n > 0 ? (size_t)n * 64 : 0; }
gfc_status gfc_render_stamps_backward(gfc_ctx*, gfc_psf*, const gfc_mix*, const gfc_galaxies*, int64_t,
                                      int, unsigned, const float*, float*, float*, void*, void*) {
  return gfc::fail(GFC_EUNSUPPORTED, "adjoint not built yet");
}
}
