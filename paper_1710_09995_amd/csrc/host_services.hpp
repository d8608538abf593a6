// Host services of the runtime (runtime.hip) that other host sources use:
// the ABI error convention and the validation of a block table.
#pragma once
#include <functional>
#include <string>

#include "../../include/cfd.h"

namespace cfd {

// Runs f; an error raised inside becomes the returned status and the text of
// cfd_last_error(NULL).  No exception leaves.
cfd_status host_guarded(const std::function<void()>& f);
// Raises an error with the given status and message (inside host_guarded).
[[noreturn]] void host_fail(cfd_status st, const std::string& msg);
// The checks cfd_create_blocks applies to block extents, and to extents and
// tables (every face of every block covered exactly once).
void host_check_dims(int nblk, const cfd_dims* dims);
void host_check_case(int nblk, const cfd_dims* dims, int nconn, const cfd_conn* conns, int nbc,
                     const cfd_bc* bcs);

}  // namespace cfd
