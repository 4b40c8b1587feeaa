// Host-side error plumbing shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdio.h>

#include <string>

#include "../../include/gmres_ir.h"

namespace gmr {

// Thread-local message returned by gmr_last_error().
std::string& last_error();

inline gmr_status fail(gmr_status s, const std::string& msg) {
  last_error() = msg;
  return s;
}

// A non-blocking stream of default priority per device, created on first use
// and owned by the library (graph capture cannot run on the legacy stream).
gmr_status library_stream(hipStream_t* out);

}  // namespace gmr
