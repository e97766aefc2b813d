// Checking builds (-DPIT_CHECK): every workgroup fills its LDS arrays with
// NaN before their first use, so a read of LDS that no thread of the
// workgroup has written makes the result NaN and fails the parity tests.
// Called at the top of a kernel by every thread of the workgroup, before any
// early return (it ends with a barrier).  Without PIT_CHECK it is empty.
#pragma once

#include <hip/hip_runtime.h>

namespace pit {

template <typename T>
__device__ __forceinline__ void poison_lds(T *p, int n)
{
#ifdef PIT_CHECK
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = (T)__builtin_nan("");
    __syncthreads();
#else
    (void)p;
    (void)n;
#endif
}

}  // namespace pit
