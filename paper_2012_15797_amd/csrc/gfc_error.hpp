// Error reporting and event logging shared by every translation unit of the
// library (no HIP): a failing call stores its message per thread for
// gfc_last_error(); with GFC_LOG=1 in the environment, errors and the
// library's events are also written to stderr as JSON lines.
#pragma once

#include <string>

#include "gfc.h"

namespace gfc {
// Records msg as this thread's last error and returns s.
gfc_status fail(gfc_status s, const std::string& msg);

// True when GFC_LOG=1 (read once).
bool log_enabled();
// Writes {"t": seconds, "event": event, <fields>} as one line to stderr;
// fields is a comma-separated list of JSON members, or empty.  Lines from
// several threads do not interleave.
void log_event(const char* event, const std::string& fields);
// s as a JSON string literal (quotes and escapes included).
std::string json_str(const std::string& s);
}  // namespace gfc
