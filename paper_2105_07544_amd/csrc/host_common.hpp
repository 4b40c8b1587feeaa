// Host-side error plumbing shared by the library's translation units.
#pragma once

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

}  // namespace gmr
