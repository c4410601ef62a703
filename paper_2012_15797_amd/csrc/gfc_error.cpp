// Per-thread error messages and status names of the C ABI (include/gfc.h).
#include <string>

#include "gfc_error.hpp"

namespace {
thread_local std::string g_last_error;
}

namespace gfc {

gfc_status fail(gfc_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

}  // namespace gfc

extern "C" {

const char* gfc_status_str(gfc_status s) {
  switch (s) {
    case GFC_OK: return "ok";
    case GFC_EINVAL: return "invalid argument";
    case GFC_EUNSUPPORTED: return "unsupported";
    case GFC_ENOMEM: return "out of memory";
    case GFC_EDEVICE: return "device error";
    case GFC_EBUSY: return "busy";
    case GFC_EREJECTED: return "rejected";
    case GFC_ETIMEOUT: return "timed out";
  }
  return "unknown status";
}

const char* gfc_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
