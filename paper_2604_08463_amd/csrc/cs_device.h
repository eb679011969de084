// Device helpers shared by the library's kernels.
#pragma once

#include "cs_internal.h"

namespace csi {

// Address-space views.  Read-only data indexed uniformly across a wavefront (work units, item
// and layout descriptors, band constants, chunk heads) is read through the constant address
// space so that it lands in scalar registers via the scalar cache; data indexed per lane goes
// through explicit global pointers instead of generic (flat) ones.
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;
template <typename T>
using gptr = const __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T *p) {
    return (cptr<T>)p;
}
template <typename T>
__device__ __forceinline__ gptr<T> as_global(const T *p) {
    return (gptr<T>)p;
}

// Load of the streamed data (read once per launch, no reuse within it): a nontemporal load, which
// on gfx950 streams through the caches without displacing what is reused (tables, label
// records, partials).
#ifndef CS_NT_LOADS
#define CS_NT_LOADS 1
#endif
template <typename T>
__device__ __forceinline__ T ld_stream(gptr<T> p) {
#if CS_NT_LOADS
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

// Streamed load through a raw buffer descriptor: voffset (per lane) + soffset (uniform) bytes,
// nontemporal like ld_stream.  kRawBufferDword3 is the descriptor's fourth dword for raw 32-bit
// data on this ISA (data format field = 32 bit, no swizzle or stride).
constexpr int kRawBufferDword3 = 0x00020000;
#if CS_NT_LOADS
constexpr int kBufAux = 2;  // nt
#else
constexpr int kBufAux = 0;
#endif
template <typename T>
__device__ __forceinline__ T ld_stream_buf(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    if constexpr (sizeof(T) == 4) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, kBufAux));
    } else {
        typedef unsigned int u2 __attribute__((ext_vector_type(2)));
        const u2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, kBufAux);
        return __longlong_as_double((long long)(((uint64_t)v.y << 32) | v.x));
    }
}

__device__ __forceinline__ uint64_t lanemask_le(int lane) {
    return lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
}

// Neumaier-compensated accumulation: s + c carries the sum.
__device__ __forceinline__ void neu_add(double &s, double &c, double v) {
    const double t = s + v;
    if (fabs(s) >= fabs(v))
        c += (s - t) + v;
    else
        c += (v - t) + s;
    s = t;
}

// Logical block index; with xcd_remap the blocks dealt round-robin to the 8 XCDs are renumbered so
// that each XCD works on one contiguous range of units (its own L2 sees neighbouring tables).
__device__ __forceinline__ int64_t logical_block(int xcd_remap) {
    const int64_t nb = gridDim.x;
    int64_t lb = blockIdx.x;
    if (xcd_remap) {
        const int64_t x = lb % kNumXcd, i = lb / kNumXcd, q = nb / kNumXcd, r = nb % kNumXcd;
        lb = x * q + (x < r ? x : r) + i;
    }
    return lb;
}

}  // namespace csi
