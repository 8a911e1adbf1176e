// Host-side kernel launch helper shared by the grid and the serving code.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <tuple>
#include <utility>

namespace sl {

// Launch through hipExtLaunchKernel so that timing events (when given) are
// part of the dispatch packet rather than extra packets on the stream.
template <typename... KArgs, typename... Args, size_t... I>
inline hipError_t launch_impl(void (*kernel)(KArgs...), dim3 grid, dim3 block, uint32_t shmem,
                       hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                       std::index_sequence<I...>, Args&&... args) {
  std::tuple<KArgs...> tup(std::forward<Args>(args)...);
  void* argv[sizeof...(KArgs) > 0 ? sizeof...(KArgs) : 1] = {
      static_cast<void*>(&std::get<I>(tup))...};
  return hipExtLaunchKernel(reinterpret_cast<const void*>(kernel), grid, block, argv, shmem,
                            s, e0, e1, 0);
}

template <typename... KArgs, typename... Args>
inline hipError_t launch(void (*kernel)(KArgs...), dim3 grid, dim3 block, uint32_t shmem,
                  hipStream_t s, hipEvent_t e0, hipEvent_t e1, Args&&... args) {
  static_assert(sizeof...(KArgs) == sizeof...(Args), "kernel argument count");
  return launch_impl(kernel, grid, block, shmem, s, e0, e1,
                     std::index_sequence_for<KArgs...>{}, std::forward<Args>(args)...);
}

}  // namespace sl
