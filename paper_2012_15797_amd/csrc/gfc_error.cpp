// Per-thread error messages, status names of the C ABI (include/gfc.h) and
// the GFC_LOG event log.
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "gfc_error.hpp"

namespace {
thread_local std::string g_last_error;
std::mutex g_log_mu;
}  // namespace

namespace gfc {

bool log_enabled() {
  static const bool on = [] {
    const char* v = std::getenv("GFC_LOG");
    return v && std::strcmp(v, "1") == 0;
  }();
  return on;
}

std::string json_str(const std::string& s) {
  std::string o = "\"";
  for (const char ch : s) {
    const unsigned char c = (unsigned char)ch;
    if (c == '"' || c == '\\') {
      o += '\\';
      o += ch;
    } else if (c < 0x20) {
      char buf[8];
      std::snprintf(buf, sizeof(buf), "\\u%04x", c);
      o += buf;
    } else {
      o += ch;
    }
  }
  return o + "\"";
}

void log_event(const char* event, const std::string& fields) {
  if (!log_enabled()) return;
  const double t = std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
  char head[96];
  std::snprintf(head, sizeof(head), "{\"t\": %.6f, \"event\": ", t);
  std::string line = head + json_str(event);
  if (!fields.empty()) line += ", " + fields;
  line += "}\n";
  std::lock_guard<std::mutex> lock(g_log_mu);
  std::fwrite(line.data(), 1, line.size(), stderr);
  std::fflush(stderr);
}

gfc_status fail(gfc_status s, const std::string& msg) {
  g_last_error = msg;
  if (log_enabled()) log_event("error", "\"status\": " + std::to_string((int)s) + ", \"message\": " + json_str(msg));
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
