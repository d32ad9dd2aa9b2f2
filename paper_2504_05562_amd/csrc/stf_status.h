// Host-side error reporting shared by the translation units of the library:
// the message of the last failed call on this thread (stf_last_error).
#pragma once

namespace stf_host {

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();
const char* last_error();

}  // namespace stf_host
