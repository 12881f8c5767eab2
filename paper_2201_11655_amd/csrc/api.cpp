// Error reporting shared by every entry point of the C ABI.
#include "vdmc_internal.h"

namespace vdmc {
namespace {
thread_local std::string t_last_error;
}
void set_error(const std::string& msg) { t_last_error = msg; }
void clear_error() { t_last_error.clear(); }
const char* last_error_cstr() { return t_last_error.c_str(); }
}  // namespace vdmc

extern "C" const char* vdmc_last_error(void) { return vdmc::last_error_cstr(); }
