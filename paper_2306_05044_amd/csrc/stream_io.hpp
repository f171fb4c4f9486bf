// Structure-of-arrays streaming I/O shared by the HBM-bound kernels.
//
// A block owns a tile of BLOCK * 4 * G consecutive elements and every lane
// handles G groups of four, read and written with 16-byte (dwordx4)
// non-temporal accesses: nothing is reused.  Each wavefront owns a contiguous
// run of 256 * G elements of its block's tile and reads it array by array, so
// the memory system sees long single-array runs (4 KiB per array per wave at
// G = 4) instead of 1 KiB pieces of nine interleaved streams; measured on the
// sampler's mix this is 6-7 % faster than lane-interleaved groups.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace capvndf {

typedef float f4 __attribute__((ext_vector_type(4)));

// Launch shape of the streaming kernels (build-time constants): threads per
// block, vec4 groups per lane, and whether loads (bit 0) and stores (bit 1)
// are non-temporal.  128 threads (two wavefronts) measured best for the VNDF
// sampler with wavefront tiles (256: within 1 %; 512: 6 % slower).
#ifndef CAPVNDF_STREAM_BLOCK
#define CAPVNDF_STREAM_BLOCK 128
#endif
#ifndef CAPVNDF_STREAM_GROUPS
#define CAPVNDF_STREAM_GROUPS 4
#endif
#ifndef CAPVNDF_STREAM_NT
#define CAPVNDF_STREAM_NT 3
#endif
// Tile layout: 1 = every wavefront owns a contiguous run of 256 * G elements
// of the tile, group g of lane l at 256 * G * wave + (g * 64 + l) * 4;
// 0 = group g of lane l at (g * BLOCK + l) * 4 (each wavefront access a 1 KiB
// piece).
#ifndef CAPVNDF_STREAM_WAVE_TILES
#define CAPVNDF_STREAM_WAVE_TILES 1
#endif

constexpr int kBlock = CAPVNDF_STREAM_BLOCK;
constexpr bool kWaveTiles = CAPVNDF_STREAM_WAVE_TILES != 0;
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

// First element of group g of this lane in the tile starting at `tile` (a
// tile holds kBlock * 4 * G elements; the groups of all lanes partition it).
template <int G, int BLOCK = kBlock, bool WT = kWaveTiles>
__device__ __forceinline__ int64_t group_start(int64_t tile, int g) {
    if (WT) {
        const int64_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        return tile + wave * 256 * G + ((int64_t)g * 64 + lane) * 4;
    }
    return tile + ((int64_t)g * BLOCK + threadIdx.x) * 4;
}

// Load the G groups of this lane from one array (the vector path's loads are
// issued array by array; groups past n are left unset, and the kernels finish
// them one element at a time).
template <int G, int BLOCK = kBlock, bool WT = kWaveTiles>
__device__ __forceinline__ void load_groups(f4 (&dst)[G], const float* __restrict__ src,
                                            int64_t tile, int64_t n) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t i0 = group_start<G, BLOCK, WT>(tile, g);
        if (i0 + 4 <= n) dst[g] = load4(src + i0);
    }
}

// Plain (cached) 16-byte store, for a kernel whose output is small next to its
// non-temporal input stream (measured faster there than a non-temporal one).
__device__ __forceinline__ void store4_cached(float* p, f4 v) { *reinterpret_cast<f4*>(p) = v; }

// Blocks for one element per lane, and for whole tiles (of G groups per lane).
inline unsigned grid_for(int64_t threads) { return (unsigned)((threads + kBlock - 1) / kBlock); }
template <int G = kGroups, int BLOCK = kBlock>
inline unsigned tiles_for(int64_t n) {
    constexpr int64_t tile = (int64_t)BLOCK * 4 * G;
    return (unsigned)((n + tile - 1) / tile);
}

// Elements per dispatch.  A dispatch's work-item count is a 32-bit number and
// the scalar paths run one element per work-item, so the element-wise entry
// points launch longer calls as consecutive slices of at most this many
// elements.  Pointers and stream positions advance by whole slices, which keeps
// each slice's 16-byte alignment and the parity of its first counter.
constexpr int64_t kSliceElems = (int64_t)1 << 31;
inline int64_t slice_len(int64_t n, int64_t off) {
    return n - off < kSliceElems ? n - off : kSliceElems;
}
template <class T>
inline T* at(T* p, int64_t off) { return p == nullptr ? p : p + off; }

}  // namespace capvndf
