// Stamp-size dispatch of the forward render.
#include "gfc_internal.hpp"
#include "gfc_launch.hpp"

namespace gfc {

gfc_status render_launch(const RenderArgs& a, int W, hipStream_t stream) {
  hipError_t e = hipErrorInvalidValue;
  switch (W) {
    case 16: e = launch_render_small<16>(a, stream); break;
    case 32: e = launch_render_small<32>(a, stream); break;
    case 64: e = launch_render_small<64>(a, stream); break;
    case 128: e = launch_render_small<128>(a, stream); break;
    case 256: e = launch_render_w256(a, stream); break;
    default: return fail(GFC_EINVAL, "unsupported stamp size");
  }
  if (e != hipSuccess) return hip_fail(e, "render launch");
  if ((a.flags & kLanczos3) && W > 64) {  // at W <= 64 the render kernel shifts while it stores
    e = launch_lanczos_shift(a, W, stream);
    if (e != hipSuccess) return hip_fail(e, "Lanczos shift launch");
  }
  return GFC_OK;
}

}  // namespace gfc
