// Task layout of the SWEEP path, shared by the host runtime and the kernel.
#pragma once

#include <stdint.h>

namespace sto {

// Rows of one reservoir (row pitch ld, element size elem_bytes) that one
// wave task of the sweep kernel covers.
int sweep_task_rows(int64_t ld, int elem_bytes);

}  // namespace sto
