// Library-internal helpers shared by api.cpp and solver.cpp.
#pragma once
#include <string>

#include "tfmm.h"

namespace tfmm {
// Number of rows (= basis functions) of a near-field matrix, 0 for NULL.
int near_rows(tfmm_near m);
// Record the detail text tfmm_last_error() returns on the calling thread.
void set_last_error(const std::string& msg);
}  // namespace tfmm
