// Library-wide C ABI helpers: version and the per-thread error message.
#include "common.hpp"

namespace mk {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
const char* get_error() { return g_last_error.c_str(); }

}  // namespace mk

extern "C" const char* mk_last_error(void) { return mk::get_error(); }

extern "C" int32_t mk_version(void) { return 100; }
