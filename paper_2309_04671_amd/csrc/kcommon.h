// Device helpers shared by the HIP kernels of this library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

namespace sp {

typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4v ld4(const float *p) { return *reinterpret_cast<const f4v *>(p); }

// Non-temporal accesses for single-use streams: they do not displace lines
// that neighbouring tiles re-read from L2.
__device__ __forceinline__ f4v ld4_nt(const float *p) {
    return __builtin_nontemporal_load(reinterpret_cast<const f4v *>(p));
}

__device__ __forceinline__ void st4_nt(float *p, f4v v) {
    __builtin_nontemporal_store(v, reinterpret_cast<f4v *>(p));
}

// Ragged row end: store the first n (1..4) values.
__device__ __forceinline__ void st_part(float *p, f4v v, int n) {
    if (n >= 4) {
        st4_nt(p, v);
    } else {
        p[0] = v[0];
        if (n > 1) p[1] = v[1];
        if (n > 2) p[2] = v[2];
    }
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Barrier that orders LDS traffic only; pending global loads stay in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Map a block index to a tile index so that each XCD receives one contiguous
// range of tiles (workgroups are dealt round-robin over the 8 XCDs, each with
// its own L2).  Bijective on [0, n) for any n.
__device__ __forceinline__ int xcd_tile(int bid, int n) {
    const int xcd = bid & 7, loc = bid >> 3, q = n >> 3, r = n & 7;
    return xcd * q + (xcd < r ? xcd : r) + loc;
}

}  // namespace sp
