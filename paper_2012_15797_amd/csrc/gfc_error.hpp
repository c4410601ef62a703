// Error reporting shared by every translation unit of the library (no HIP):
// a failing call stores its message per thread for gfc_last_error().
#pragma once

#include <string>

#include "gfc.h"

namespace gfc {
// Records msg as this thread's last error and returns s.
gfc_status fail(gfc_status s, const std::string& msg);
}  // namespace gfc
