// vmc_error.hpp -- error reporting shared by the C ABI units: sets the
// calling thread's message returned by vmc_last_error() and returns `code`.
#pragma once

namespace vmc {
int set_error(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
}  // namespace vmc
