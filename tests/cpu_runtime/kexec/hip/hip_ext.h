// CPU execution of the library's kernels: hipExtLaunchKernelGGL comes with
// the replacement <hip/hip_runtime.h>.
#pragma once
#include <hip/hip_runtime.h>
