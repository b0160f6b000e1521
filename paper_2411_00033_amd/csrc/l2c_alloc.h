// l2c_alloc.h -- the library's device and pinned host allocations.
//
// Every allocation goes through these, so that the allocation-failure hook of the ABI
// (leg2cheb_debug_alloc_hook) can fail any one of them and count what is still held.
// dev_free / host_free accept null.  Implemented in l2c_api.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace l2c {

hipError_t dev_alloc_raw(void **ptr, size_t bytes);
template <typename T>
hipError_t dev_alloc(T **ptr, size_t bytes)
{
    return dev_alloc_raw((void **)ptr, bytes);
}
void dev_free(const void *ptr);
hipError_t host_alloc(void **ptr, size_t bytes, unsigned flags = hipHostMallocDefault);
void host_free(void *ptr);

}  // namespace l2c
