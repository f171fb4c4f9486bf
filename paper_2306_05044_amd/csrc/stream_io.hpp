// Structure-of-arrays streaming I/O shared by the HBM-bound kernels.
//
// A block owns a tile of kBlock * 4 * kGroups consecutive elements; lane l
// handles kGroups groups of four, group g starting at tile + (g * kBlock + l)
// * 4, so every wavefront access is a contiguous 1 KiB per array, read and
// written with 16-byte (dwordx4) accesses that are non-temporal: nothing is
// reused.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace capvndf {

typedef float f4 __attribute__((ext_vector_type(4)));

// Launch shape of the streaming kernels (build-time constants): threads per
// block, vec4 groups per lane, and whether loads (bit 0) and stores (bit 1)
// are non-temporal.
#ifndef CAPVNDF_STREAM_BLOCK
#define CAPVNDF_STREAM_BLOCK 256
#endif
#ifndef CAPVNDF_STREAM_GROUPS
#define CAPVNDF_STREAM_GROUPS 4
#endif
#ifndef CAPVNDF_STREAM_NT
#define CAPVNDF_STREAM_NT 3
#endif
constexpr int kBlock = CAPVNDF_STREAM_BLOCK;
constexpr int kGroups = CAPVNDF_STREAM_GROUPS;
constexpr int64_t kTile = (int64_t)kBlock * 4 * kGroups;

__device__ __forceinline__ f4 load4(const float* p) {
    if (CAPVNDF_STREAM_NT & 1) return __builtin_nontemporal_load(reinterpret_cast<const f4*>(p));
    return *reinterpret_cast<const f4*>(p);
}
__device__ __forceinline__ void store4(float* p, f4 v) {
    if (CAPVNDF_STREAM_NT & 2)
        __builtin_nontemporal_store(v, reinterpret_cast<f4*>(p));
    else
        *reinterpret_cast<f4*>(p) = v;
}

// Plain (cached) 16-byte store, for a kernel whose output is small next to its
// non-temporal input stream (measured faster there than a non-temporal one).
__device__ __forceinline__ void store4_cached(float* p, f4 v) { *reinterpret_cast<f4*>(p) = v; }

// Blocks for one element per lane, and for whole tiles (of G groups per lane).
inline unsigned grid_for(int64_t threads) { return (unsigned)((threads + kBlock - 1) / kBlock); }
template <int G = kGroups>
inline unsigned tiles_for(int64_t n) {
    constexpr int64_t tile = (int64_t)kBlock * 4 * G;
    return (unsigned)((n + tile - 1) / tile);
}

}  // namespace capvndf
