// Global-address-space views of device pointers.
#pragma once

namespace ircur {

// Pointers that come out of argument tables in memory are generic to the
// compiler, and generic (flat) accesses also hold up the waits for LDS
// results.  gp() gives such a pointer its global address space.
typedef __attribute__((address_space(1))) double gdouble;
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gp(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}

}  // namespace ircur
