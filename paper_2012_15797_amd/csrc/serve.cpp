// Serving scheduler (placeholder until the continuous-batching server lands).
#include "gfc_internal.hpp"

extern "C" {
gfc_status gfc_server_create(gfc_ctx*, size_t, int, int64_t, gfc_server**) {
  return gfc::fail(GFC_EUNSUPPORTED, "server not built yet");
}
gfc_status gfc_server_submit(gfc_server*, const gfc_request*, uint64_t*) { return GFC_EUNSUPPORTED; }
gfc_status gfc_server_poll(gfc_server*, uint64_t, int*, const float**, gfc_status*) { return GFC_EUNSUPPORTED; }
gfc_status gfc_server_wait(gfc_server*, uint64_t, int, const float**) { return GFC_EUNSUPPORTED; }
gfc_status gfc_server_release(gfc_server*, uint64_t) { return GFC_EUNSUPPORTED; }
gfc_status gfc_server_stats(gfc_server*, double*, double*, double*, double*, uint64_t*, uint64_t*) {
  return GFC_EUNSUPPORTED;
}
gfc_status gfc_server_destroy(gfc_server*) { return GFC_EUNSUPPORTED; }
}
