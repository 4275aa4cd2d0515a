// Error reporting shared by the library's host code: api_fail records the
// message for ppm_last_error and returns the status code.  No HIP types, so
// host-only sources (the OGIP reader) build with any C++ compiler.
#pragma once

namespace ppm {

int api_fail(int code, const char *msg);   // sets ppm_last_error, returns code

}  // namespace ppm
