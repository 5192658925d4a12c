// Loads through the global address space.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace sd7 {

// Element i of a device array, loaded through the global address space.
// Pointers taken from the frame table are generic, and generic (flat) loads
// may alias LDS, which keeps the compiler from moving them past LDS stores or
// batching them ahead of those stores.
template <class T>
__device__ __forceinline__ T gload(const T* p, size_t i)
{
    return ((const __attribute__((address_space(1))) T*)p)[i];
}

}  // namespace sd7
