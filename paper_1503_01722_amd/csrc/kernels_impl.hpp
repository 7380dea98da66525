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
    if (a.src_order)
        hipLaunchKernelGGL(source_ordered_kernel<R>, dim3(grid), dim3(block), 0,
                           (hipStream_t)stream, a);
    else
        hipLaunchKernelGGL(source_kernel<R>, dim3(grid), dim3(block), 0, (hipStream_t)stream, a);
    return detail::launch_status();
}

template <typename R>
int Launch<R>::source_groups(const KernelArgs<R>& a, int grid, void* stream)
{
    hipLaunchKernelGGL(source_group_kernel<R>, dim3(grid), dim3(256), 0, (hipStream_t)stream, a);
    return detail::launch_status();
}

// Allow more than 64 KB of dynamic LDS where the tables need it (done before
// any launch, outside stream capture).
template <typename R>
int Launch<R>::prepare(size_t lds_ph, size_t lds_el, bool gtab)
{
    auto raise = [](const void* f, size_t lds) {
        return lds > 65536 && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                  int(lds)) != hipSuccess;
    };
    if (gtab)
        return raise((const void*)photon_kernel<R, true, false>, lds_ph) ||
                       raise((const void*)photon_kernel<R, true, true>, lds_ph) ||
                       raise((const void*)electron_kernel<R, false, true>, lds_el) ||
                       raise((const void*)electron_kernel<R, true, true>, lds_el)
                   ? -1
                   : 0;
    return raise((const void*)photon_kernel<R, false, false>, lds_ph) ||
                   raise((const void*)photon_kernel<R, false, true>, lds_ph) ||
                   raise((const void*)electron_kernel<R, false, false>, lds_el) ||
                   raise((const void*)electron_kernel<R, true, false>, lds_el)
               ? -1
               : 0;
}

template <typename R>
int Launch<R>::photon(const KernelArgs<R>& a, int grid, int block, size_t lds, bool gtab,
                      bool cells, void* stream)
{
    const hipStream_t s = (hipStream_t)stream;
    if (gtab && cells)
        hipLaunchKernelGGL((photon_kernel<R, true, true>), dim3(grid), dim3(block), lds, s, a);
    else if (gtab)
        hipLaunchKernelGGL((photon_kernel<R, true, false>), dim3(grid), dim3(block), lds, s, a);
    else if (cells)
        hipLaunchKernelGGL((photon_kernel<R, false, true>), dim3(grid), dim3(block), lds, s, a);
    else
        hipLaunchKernelGGL((photon_kernel<R, false, false>), dim3(grid), dim3(block), lds, s, a);
    return detail::launch_status();
}

template <typename R>
int Launch<R>::electron(const KernelArgs<R>& a, int grid, int block, size_t lds, bool fixed,
                        bool gtab, void* stream)
{
    const hipStream_t s = (hipStream_t)stream;
    if (fixed && gtab)
        hipLaunchKernelGGL((electron_kernel<R, true, true>), dim3(grid), dim3(block), lds, s, a);
    else if (fixed)
        hipLaunchKernelGGL((electron_kernel<R, true, false>), dim3(grid), dim3(block), lds, s, a);
    else if (gtab)
        hipLaunchKernelGGL((electron_kernel<R, false, true>), dim3(grid), dim3(block), lds, s, a);
    else
        hipLaunchKernelGGL((electron_kernel<R, false, false>), dim3(grid), dim3(block), lds, s,
                           a);
    return detail::launch_status();
}

template <typename R>
int Launch<R>::sample(const KernelArgs<R>& a, const SampleArgs& sa, double* out, uint32_t* words,
                      void* stream)
{
    hipLaunchKernelGGL(sample_kernel<R>, dim3((sa.n + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, a, sa, out, words);
    return detail::launch_status();
}

}  // namespace omc
