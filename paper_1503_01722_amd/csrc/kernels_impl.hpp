// kernels_impl.hpp -- host launchers for one transport precision R. Included by
// one translation unit per precision (FP32 production, FP64 parity).
#pragma once

#include "device.hpp"

namespace omc {

namespace detail {
inline int launch_status()
{
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
}  // namespace detail

template <typename R>
int Launch<R>::source(const KernelArgs<R>& a, int grid, int block, void* stream)
{
    hipLaunchKernelGGL(source_kernel<R>, dim3(grid), dim3(block), 0, (hipStream_t)stream, a);
    return detail::launch_status();
}

// Allow more than 64 KB of dynamic LDS where the tables need it (done before
// any launch, outside stream capture).
template <typename R>
int Launch<R>::prepare(size_t lds_ph, size_t lds_el)
{
    if (lds_ph > 65536 &&
        hipFuncSetAttribute((const void*)photon_kernel<R>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_ph)) != hipSuccess)
        return -1;
    if (lds_el > 65536 &&
        (hipFuncSetAttribute((const void*)electron_kernel<R, false>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_el)) != hipSuccess ||
         hipFuncSetAttribute((const void*)electron_kernel<R, true>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_el)) != hipSuccess))
        return -1;
    return 0;
}

template <typename R>
int Launch<R>::photon(const KernelArgs<R>& a, int grid, int block, size_t lds, void* stream)
{
    hipLaunchKernelGGL(photon_kernel<R>, dim3(grid), dim3(block), lds, (hipStream_t)stream, a);
    return detail::launch_status();
}

template <typename R>
int Launch<R>::electron(const KernelArgs<R>& a, int grid, int block, size_t lds, bool fixed,
                        void* stream)
{
    if (fixed)
        hipLaunchKernelGGL((electron_kernel<R, true>), dim3(grid), dim3(block), lds,
                           (hipStream_t)stream, a);
    else
        hipLaunchKernelGGL((electron_kernel<R, false>), dim3(grid), dim3(block), lds,
                           (hipStream_t)stream, a);
    return detail::launch_status();
}

}  // namespace omc
