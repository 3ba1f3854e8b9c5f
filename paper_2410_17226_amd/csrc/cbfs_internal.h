// Internal declarations shared by the translation units of libcbfs.
#pragma once
#include <cstdint>

#include <hip/hip_runtime.h>

#include "cbfs.h"

namespace cbfs {

// Records `msg` as the calling thread's last error and returns `s`.
cbfs_status fail(cbfs_status s, const char *msg);
// Records a formatted HIP failure ("<what>: <hip error string>") and returns CBFS_E_HIP.
cbfs_status hip_fail(const char *what, int hip_error);
// Kernel timing hooks (no-ops unless cbfs_profile_enable(1) was called).
void prof_begin(int kind, hipStream_t st, void **token);
void prof_end(void *token);

}  // namespace cbfs
