// Kernel launch with optional timing events taken by the dispatch itself.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

namespace ca {

// With `start` set, hipExtLaunchKernelGGL records start and stop at the
// kernel's own begin and end (no marker packets around it, so the elapsed
// time is the kernel's duration, as a kernel trace reports it); otherwise a
// plain launch.
template <typename K, typename... Args>
inline void launch_maybe_timed(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s,
                               hipEvent_t start, hipEvent_t stop, Args... args)
{
    if (start)
        hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, s, start, stop, 0u, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
}

}  // namespace ca
