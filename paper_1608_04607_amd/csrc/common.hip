// Error reporting shared by all entry points.
#include <string>

#include "dfm_internal.h"

namespace dfm {
namespace {
thread_local std::string g_last_error;
}
void set_error(const std::string &msg) { g_last_error = msg; }
}  // namespace dfm

extern "C" const char *dfm_last_error(void) { return dfm::g_last_error.c_str(); }
