// Directional-albedo estimator kernels: forward (two sums from one stream),
// pathwise adjoint, the batched persistent forward+adjoint kernel and the
// fixed-order finishing pass, plus their C entry points.
//
// Work decomposition: a cell (or job) of N samples is N/2 Philox pairs, cut
// into chunks of block * pairs_per_thread pairs (or 64 * pairs_per_thread when
// a batch gives chunks to single wavefronts).  The owner reduces a chunk to a
// compensated partial (lane TwoSum accumulators -> wavefront DPP/permute
// butterfly -> LDS across waves); the finishing pass merges a cell's chunk
// partials in chunk order.  No atomics anywhere, so every result is bitwise
// reproducible.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "albedo_math.hpp"
#include "common.hpp"

namespace capvndf {
namespace {

constexpr int kLutBlock = 256;
constexpr int kLutPairsPerThread = 32;
constexpr uint64_t kLutChunkPairs = (uint64_t)kLutBlock * kLutPairsPerThread;
constexpr int kGroup = 8;  // pairs summed plainly before each TwoSum fold
// Unroll depth of the adjoint's pair loop and the waves per SIMD the
// adjoint kernels are compiled for (build-time tuning constants).  Seven
// resident waves beat the compiler's default register budget (five waves) by
// about 8 % on gfx950, even though a few loop-invariant values then spill;
// the table's gradient-only (recompute) kernel runs 1 % faster at six (the
// value + gradient kernel 5 % slower, the batch kernels 0-2 % slower).
#ifndef CAPVNDF_ADJ_UNROLL
#define CAPVNDF_ADJ_UNROLL 1
#endif
#ifndef CAPVNDF_ADJ_WAVES
#define CAPVNDF_ADJ_WAVES 7
#endif
#ifndef CAPVNDF_ADJ_GRAD_WAVES
#define CAPVNDF_ADJ_GRAD_WAVES 6
#endif
constexpr int kFinishBlock = 256;

// ---------------------------------------------------------------------------
// Reductions.
// ---------------------------------------------------------------------------
// Wavefront reduction of compensated pairs.  Four DPP steps combine the 16
// lanes of each row in registers (quad xor 1, quad xor 2, half-row mirror, row
// mirror; lanes that exchanged then hold identical bits, since TwoSum's error
// term does not depend on the operand order), and two lane permutes across
// rows (xor 16, xor 32) finish the butterfly.  Every lane returns the wave
// total; the tree is fixed, so the result is reproducible.  Must be reached
// by all 64 lanes.  (Reading the four row totals with readlane instead of the
// last two permutes measured 12 % slower for the adjoint kernels: the
// compiler schedules their sample loop worse.)
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ Comp dpp_merge(const Comp& v) {
    return comp_merge(v, Comp{dpp_mov<CTRL>(v.s), dpp_mov<CTRL>(v.c)});
}
__device__ __forceinline__ Comp wave_reduce(Comp v) {
    v = dpp_merge<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v = dpp_merge<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v = dpp_merge<0x141>(v);  // row_half_mirror
    v = dpp_merge<0x140>(v);  // row_mirror
#pragma unroll
    for (int off = 16; off <= 32; off <<= 1) {
        const Comp o{__shfl_xor(v.s, off, 64), __shfl_xor(v.c, off, 64)};
        v = comp_merge(v, o);
    }
    return v;
}

// Reduce NACC compensated accumulators over the block and store them as
// (s, c) pairs at dst[0 .. 2*NACC).  Must be reached by every thread.
template <int NACC, int BLOCK>
__device__ __forceinline__ void block_reduce_store(Comp (&acc)[NACC], float* __restrict__ dst) {
    __shared__ Comp red[BLOCK / 64][NACC];
#pragma unroll
    for (int a = 0; a < NACC; ++a) acc[a] = wave_reduce(acc[a]);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int a = 0; a < NACC; ++a) red[wave][a] = acc[a];
    }
    __syncthreads();
    if (threadIdx.x < NACC) {
        const int a = threadIdx.x;
        Comp r = red[0][a];
        for (int w = 1; w < BLOCK / 64; ++w) r = comp_merge(r, red[w][a]);
        dst[2 * a] = r.s;
        dst[2 * a + 1] = r.c;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Per-thread sample loops over pairs [pbeg, pend) with stride BLOCK.
// ---------------------------------------------------------------------------
template <int STRIDE>
__device__ __forceinline__ void pairs_fwd(const CellConst& c, uint64_t pbeg, uint64_t pend,
                                          uint64_t nsamples, uint32_t unit, uint32_t k0,
                                          uint32_t k1, Comp (&acc)[2], uint32_t lane = threadIdx.x) {
    for (uint64_t p0 = pbeg + lane; p0 < pend; p0 += (uint64_t)STRIDE * kGroup) {
        float sg = 0.0f, sgm = 0.0f;
#pragma unroll 2
        for (int j = 0; j < kGroup; ++j) {
            const uint64_t p = p0 + (uint64_t)j * STRIDE;
            if (p < pend) {
                const Words w = philox_pair(p, unit, kTagAlbedo, k0, k1);
                const FwdTerm t0 = albedo_fwd(c, unit24(w.w0), unit24(w.w1));
                sg += t0.g;
                sgm = __builtin_fmaf(t0.g, t0.m5, sgm);
                if (2 * p + 1 < nsamples) {
                    const FwdTerm t1 = albedo_fwd(c, unit24(w.w2), unit24(w.w3));
                    sg += t1.g;
                    sgm = __builtin_fmaf(t1.g, t1.m5, sgm);
                }
            }
        }
        comp_add(acc[0], sg);
        comp_add(acc[1], sgm);
    }
}

// The table's forward loop over one chunk: pairs base + off for off < len,
// a pair's second sample existing for off < sec (2 p + 1 < n, i.e.
// p < n / 2).  base is a multiple of kLutChunkPairs and len at most
// kLutChunkPairs, so offsets and bounds fit 32 bits and the pair index
// base + off is base | off: the same pairs in the same order as pairs_fwd,
// with no 64-bit index arithmetic per pair.  Measured on gfx950: the
// table's forward kernel 1.4 % faster; the same form in the table's
// adjoint kernel within 1 % either way from box to box, and in the batch's
// persistent kernels (chunks at any pair offset, so a 64-bit add per pair)
// 5 % slower, so those keep pairs_adj and pairs_fwd.
struct Chunk {
    uint32_t lo, hi;  // base
    uint32_t len, sec;
};

__device__ __forceinline__ Chunk table_chunk(int64_t k, uint64_t npairs, uint64_t n) {
    const uint64_t pbeg = (uint64_t)k * kLutChunkPairs;
    const uint64_t pend = std::min(pbeg + kLutChunkPairs, npairs);
    const uint64_t full = std::min(std::max(n / 2, pbeg), pend);
    return Chunk{(uint32_t)pbeg, (uint32_t)(pbeg >> 32), (uint32_t)(pend - pbeg),
                 (uint32_t)(full - pbeg)};
}

template <int STRIDE>
__device__ __forceinline__ void chunk_fwd(const CellConst& c, const Chunk& ck, uint32_t unit,
                                          uint32_t k0, uint32_t k1, Comp (&acc)[2]) {
    for (uint32_t off0 = threadIdx.x; off0 < ck.len; off0 += (uint32_t)STRIDE * kGroup) {
        float sg = 0.0f, sgm = 0.0f;
#pragma unroll 2
        for (int j = 0; j < kGroup; ++j) {
            const uint32_t off = off0 + (uint32_t)j * STRIDE;
            if (off < ck.len) {
                const Words w = philox4x32_10(ck.lo | off, unit, kTagAlbedo, ck.hi, k0, k1);
                const FwdTerm t0 = albedo_fwd(c, unit24(w.w0), unit24(w.w1));
                sg += t0.g;
                sgm = __builtin_fmaf(t0.g, t0.m5, sgm);
                if (off < ck.sec) {
                    const FwdTerm t1 = albedo_fwd(c, unit24(w.w2), unit24(w.w3));
                    sg += t1.g;
                    sgm = __builtin_fmaf(t1.g, t1.m5, sgm);
                }
            }
        }
        comp_add(acc[0], sg);
        comp_add(acc[1], sgm);
    }
}

// ---------------------------------------------------------------------------
// Horizon records.  albedo_adj flags, with a margin >= 0, the samples whose
// FP32 reflection lies within rounding of the horizon or whose conditioning
// is too poor for FP32 (a few in 10^5).  The adjoint loops keep per lane the
// largest margin of its samples; the owner of each partial (a table slot's
// block, a batch chunk's block or wavefront) then stores one 64-bit mask of
// its flagged lanes per wavefront, its record.  The fix pass walks the
// pairs of the flagged lanes again, evaluates their flagged samples in
// double precision and adds t64 - t32 to the owner's partial in a fixed
// order.  The sample loops so carry one float and hold no call: a call
// there, even one never taken, made them 1.4x to 2.9x slower on gfx950.
// ---------------------------------------------------------------------------

// Bytes of the records of nowners owners of nwords wavefronts.
__host__ __device__ inline size_t rec_bytes(int64_t nowners, int nwords) {
    return (size_t)nowners * (size_t)nwords * sizeof(uint64_t);
}

// Record of a block owner: rec[w] = flags of wavefront w.
__device__ __forceinline__ void store_flags_block(float margin, uint64_t* __restrict__ rec) {
    const uint64_t m = __ballot(margin >= 0.0f);
    if ((threadIdx.x & 63) == 0) rec[threadIdx.x >> 6] = m;
}

// Record of a wavefront owner.  Must be reached by all 64 lanes.
__device__ __forceinline__ void store_flags_wave(float margin, uint32_t lane,
                                                 uint64_t* __restrict__ rec) {
    const uint64_t m = __ballot(margin >= 0.0f);
    if (lane == 0) rec[0] = m;
}

// Adjoint loop: sums w and the derivatives over the lane's pairs.  Each
// group of kGroup pairs sums the direct derivatives and the adjoint of ws
// plainly, chains the ws adjoint into (alpha_x, alpha_y, theta_o) (ws_chain
// is linear, and its constants are the cell's) and folds the four results
// into compensated sums: out = {w, gax, gay, gth}.  margin is raised to the
// largest margin of the lane's samples (horizon records).
template <int STRIDE>
__device__ __forceinline__ void pairs_adj(const CellConst& c, float f0, uint64_t pbeg,
                                          uint64_t pend, uint64_t nsamples, uint32_t unit,
                                          uint32_t k0, uint32_t k1, Comp (&out)[4], float& margin,
                                          uint32_t lane = threadIdx.x) {
    Comp acc[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) acc[a] = Comp{0.0f, 0.0f};
    for (uint64_t p0 = pbeg + lane; p0 < pend; p0 += (uint64_t)STRIDE * kGroup) {
        float part[7] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll CAPVNDF_ADJ_UNROLL
        for (int j = 0; j < kGroup; ++j) {
            const uint64_t p = p0 + (uint64_t)j * STRIDE;
            if (p < pend) {
                const Words w = philox_pair(p, unit, kTagAlbedo, k0, k1);
                const AdjTerm t0 = albedo_adj(c, f0, unit24(w.w0), unit24(w.w1));
                part[0] += t0.w; part[1] += t0.dax; part[2] += t0.day; part[3] += t0.dth;
                part[4] += t0.dwsx; part[5] += t0.dwsy; part[6] += t0.dzs;
                float f = t0.margin;
                if (2 * p + 1 < nsamples) {
                    const AdjTerm t1 = albedo_adj(c, f0, unit24(w.w2), unit24(w.w3));
                    part[0] += t1.w; part[1] += t1.dax; part[2] += t1.day; part[3] += t1.dth;
                    part[4] += t1.dwsx; part[5] += t1.dwsy; part[6] += t1.dzs;
                    f = fmaxf(f, t1.margin);
                }
                margin = fmaxf(margin, f);
            }
        }
        ws_chain(c, part[4], part[5], part[6], part[1], part[2], part[3]);
#pragma unroll
        for (int a = 0; a < 4; ++a) comp_add(acc[a], part[a]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) out[a] = acc[a];
}

// ---------------------------------------------------------------------------
// Table estimators: per-cell sample counts, cells cut into slots.
//
// Cell c has N_c samples (its own count, read from device memory), i.e.
// ceil(ceil(N_c / 2) / kLutChunkPairs) chunks.  A launch gives every cell
// `slots` consecutive blocks; slot s of a cell handles the cell's chunks
// s, s + slots, s + 2 slots, ... into one compensated partial, and the
// finishing pass merges the cell's first min(slots, chunks) partials in slot
// order.  A slot beyond the cell's chunk count returns at once.  The slot
// count is a host choice (enough blocks to fill the chip, capped by the
// workspace), so no device-side table or scan is needed and a workspace
// depends only on the cell count.
// ---------------------------------------------------------------------------
constexpr int64_t kMaxSamples = (int64_t)1 << 40;

__host__ __device__ inline int64_t cell_chunks(int64_t n) {
    if (n <= 0 || n >= kMaxSamples) return 0;
    const uint64_t npairs = ((uint64_t)n + 1) / 2;
    return (int64_t)((npairs + kLutChunkPairs - 1) / kLutChunkPairs);
}

// The part of a launch that block b works on.
struct SlotWork {
    int64_t cell;    // cell index within the call
    int64_t nchunks; // chunks of the cell
    uint64_t n;      // its sample count
    int32_t slot;
};

__device__ __forceinline__ SlotWork slot_work(const int64_t* __restrict__ nsamp, int32_t slots) {
    SlotWork w;
    const int64_t b = blockIdx.x;
    w.cell = b / slots;
    w.slot = (int32_t)(b - w.cell * slots);
    const int64_t n = nsamp[w.cell];
    w.nchunks = cell_chunks(n);
    w.n = w.nchunks > 0 ? (uint64_t)n : 0;
    return w;
}

// MODE 0: two sums (G2/G1 and G2/G1 (1 - wo.h)^5) for albedo_estimate;
// MODE 1: one sum of F G2/G1 with the cell's F0.
template <int MODE>
__global__ __launch_bounds__(kLutBlock) void k_albedo_fwd(
    const float* __restrict__ wox, const float* __restrict__ woy, const float* __restrict__ woz,
    const float* __restrict__ ax, const float* __restrict__ ay, const float* __restrict__ f0p,
    const int64_t* __restrict__ nsamp, int32_t slots, uint32_t unit_base, uint32_t k0,
    uint32_t k1, float* __restrict__ partial) {
    constexpr int NACC = MODE == 0 ? 2 : 1;
    const SlotWork sw = slot_work(nsamp, slots);
    if (sw.slot >= sw.nchunks) return;  // the same for the whole block
    const int64_t cell = sw.cell;
    const CellConst c = cell_setup(wox[cell], woy[cell], woz[cell], ax[cell], ay[cell]);
    Comp acc[2] = {Comp{0.0f, 0.0f}, Comp{0.0f, 0.0f}};
    const uint64_t npairs = (sw.n + 1) / 2;
    if (c.ok)
        for (int64_t k = sw.slot; k < sw.nchunks; k += slots)
            chunk_fwd<kLutBlock>(c, table_chunk(k, npairs, sw.n), unit_base + (uint32_t)cell, k0,
                                 k1, acc);
    float* dst = partial + (int64_t)blockIdx.x * 2 * NACC;
    if (MODE == 0) {
        block_reduce_store<2, kLutBlock>(acc, dst);
    } else {
        // A(F0) = F0 S1 + (1 - F0) S5, folded per lane
        const float f0 = f0p ? f0p[cell] : 1.0f;
        const float a1 = acc[0].s + acc[0].c, a5 = acc[1].s + acc[1].c;
        Comp w[1] = {Comp{__builtin_fmaf(f0, a1, (1.0f - f0) * a5), 0.0f}};
        block_reduce_store<1, kLutBlock>(w, dst);
    }
}

// Adjoint of A(F0); WITH_VALUE also reduces the value itself (4 sums: A,
// dA/d alpha_x, dA/d alpha_y, dA/d theta_o), otherwise the 3 gradient sums.
// Block b also writes its horizon record at rec[4 b .. 4 b + 4).
#define CAPVNDF_ADJ_ATTR __attribute__((amdgpu_waves_per_eu(CAPVNDF_ADJ_WAVES)))
template <bool WITH_VALUE>
__global__ __launch_bounds__(kLutBlock) __attribute__((amdgpu_waves_per_eu(
    WITH_VALUE ? CAPVNDF_ADJ_WAVES : CAPVNDF_ADJ_GRAD_WAVES))) void k_albedo_adj(
    const float* __restrict__ wox, const float* __restrict__ woy, const float* __restrict__ woz,
    const float* __restrict__ ax, const float* __restrict__ ay, const float* __restrict__ f0p,
    const int64_t* __restrict__ nsamp, int32_t slots, uint32_t unit_base, uint32_t k0,
    uint32_t k1, float* __restrict__ partial, uint64_t* __restrict__ rec) {
    const SlotWork sw = slot_work(nsamp, slots);
    if (sw.slot >= sw.nchunks) return;
    const int64_t cell = sw.cell;
    const CellConst c = cell_setup(wox[cell], woy[cell], woz[cell], ax[cell], ay[cell]);
    const float f0 = f0p ? f0p[cell] : 1.0f;
    Comp out[4] = {Comp{0.0f, 0.0f}, Comp{0.0f, 0.0f}, Comp{0.0f, 0.0f}, Comp{0.0f, 0.0f}};
    float margin = -1.0f;
    const uint64_t npairs = (sw.n + 1) / 2;
    if (c.ok) {
        // one sweep per chunk of the slot; the pathwise sums of successive
        // chunks are added in chunk order (each already compensated)
        for (int64_t k = sw.slot; k < sw.nchunks; k += slots) {
            const uint64_t pbeg = (uint64_t)k * kLutChunkPairs;
            const uint64_t pend = std::min(pbeg + kLutChunkPairs, npairs);
            Comp part[4];
            pairs_adj<kLutBlock>(c, f0, pbeg, pend, sw.n, unit_base + (uint32_t)cell, k0, k1,
                                 part, margin);
#pragma unroll
            for (int a = 0; a < 4; ++a) out[a] = comp_merge(out[a], part[a]);
        }
    }
    float* dst = partial + (int64_t)blockIdx.x * (WITH_VALUE ? 8 : 6);
    if (WITH_VALUE) {
        block_reduce_store<4, kLutBlock>(out, dst);
    } else {
        Comp g[3] = {out[1], out[2], out[3]};
        block_reduce_store<3, kLutBlock>(g, dst);
    }
    store_flags_block(margin, rec + (int64_t)blockIdx.x * (kLutBlock / 64));
}

// Direct illumination: one sum of F G2/G1 L(wl) per cell, NL lobes.
template <int NL>
__global__ __launch_bounds__(kLutBlock) void k_radiance(
    const float* __restrict__ wox, const float* __restrict__ woy, const float* __restrict__ woz,
    const float* __restrict__ ax, const float* __restrict__ ay, const float* __restrict__ f0p,
    const float* __restrict__ lobep, const int64_t* __restrict__ nsamp, int32_t slots,
    uint32_t k0, uint32_t k1, float* __restrict__ partial) {
    const SlotWork sw = slot_work(nsamp, slots);
    if (sw.slot >= sw.nchunks) return;
    const int64_t cell = sw.cell;
    const CellConst c = cell_setup(wox[cell], woy[cell], woz[cell], ax[cell], ay[cell]);
    const float f0 = f0p ? f0p[cell] : 1.0f;
    const Lobes<NL> lobes = load_lobes<NL>(lobep);
    Comp acc[1] = {Comp{0.0f, 0.0f}};
    const uint64_t npairs = (sw.n + 1) / 2;
    if (c.ok) {
        const uint32_t unit = (uint32_t)cell;
        for (int64_t k = sw.slot; k < sw.nchunks; k += slots) {
            const uint64_t pbeg = (uint64_t)k * kLutChunkPairs;
            const uint64_t pend = std::min(pbeg + kLutChunkPairs, npairs);
            for (uint64_t p0 = pbeg + threadIdx.x; p0 < pend; p0 += (uint64_t)kLutBlock * kGroup) {
                float part = 0.0f;
                // fully unrolled: 1.7 % faster than by 2 on gfx950 (the
                // forward loop above is fastest by 2)
#pragma unroll
                for (int j = 0; j < kGroup; ++j) {
                    const uint64_t p = p0 + (uint64_t)j * kLutBlock;
                    if (p < pend) {
                        const Words w = philox_pair(p, unit, kTagAlbedo, k0, k1);
                        part += radiance_term(c, f0, lobes, unit24(w.w0), unit24(w.w1));
                        if (2 * p + 1 < sw.n)
                            part += radiance_term(c, f0, lobes, unit24(w.w2), unit24(w.w3));
                    }
                }
                comp_add(acc[0], part);
            }
        }
    }
    block_reduce_store<1, kLutBlock>(acc, partial + (int64_t)blockIdx.x * 2);
}

// ---------------------------------------------------------------------------
// Batched persistent kernels.  Each chunk is (job, pair range) and owns one
// slot of `partial`, so results do not depend on which block or wavefront
// processes it.  Static scheduling: owner o walks its precomputed range
// [owner_chunks[o], owner_chunks[o+1]) (balanced by sample count).  Dynamic
// scheduling: owners take the next chunk index from a device counter (reset
// to 0 before every launch) until it passes nchunks, so every owner exits.
// ---------------------------------------------------------------------------
template <int BLOCK, bool GRAD>
__device__ __forceinline__ void batch_chunk_block(
    int32_t ch, const float* __restrict__ wox, const float* __restrict__ woy,
    const float* __restrict__ woz, const float* __restrict__ ax, const float* __restrict__ ay,
    const float* __restrict__ f0p, const int64_t* __restrict__ nsamp,
    const int32_t* __restrict__ chunk_job, const int64_t* __restrict__ chunk_pbeg,
    const int64_t* __restrict__ chunk_pend, uint32_t k0, uint32_t k1,
    float* __restrict__ partial, uint64_t* __restrict__ rec) {
    const int32_t j = chunk_job[ch];
    const CellConst c = cell_setup(wox[j], woy[j], woz[j], ax[j], ay[j]);
    const float f0 = f0p ? f0p[j] : 1.0f;
    const uint64_t n = (uint64_t)nsamp[j];
    const uint64_t pbeg = (uint64_t)chunk_pbeg[ch];
    const uint64_t pend = (uint64_t)chunk_pend[ch];
    if (GRAD) {
        Comp out[4] = {Comp{0.0f, 0.0f}, Comp{0.0f, 0.0f}, Comp{0.0f, 0.0f}, Comp{0.0f, 0.0f}};
        float margin = -1.0f;
        if (c.ok) pairs_adj<BLOCK>(c, f0, pbeg, pend, n, (uint32_t)j, k0, k1, out, margin);
        block_reduce_store<4, BLOCK>(out, partial + (int64_t)ch * 8);
        store_flags_block(margin, rec + (int64_t)ch * (BLOCK / 64));
    } else {
        Comp acc[2] = {Comp{0.0f, 0.0f}, Comp{0.0f, 0.0f}};
        if (c.ok) pairs_fwd<BLOCK>(c, pbeg, pend, n, (uint32_t)j, k0, k1, acc);
        // A(F0) = F0 S1 + (1 - F0) S5, folded per chunk
        const float a1 = acc[0].s + acc[0].c, a5 = acc[1].s + acc[1].c;
        Comp w[1] = {Comp{__builtin_fmaf(f0, a1, (1.0f - f0) * a5), 0.0f}};
        block_reduce_store<1, BLOCK>(w, partial + (int64_t)ch * 2);
    }
}

template <bool GRAD>
__device__ __forceinline__ void batch_chunk_wave(
    int32_t ch, uint32_t lane, const float* __restrict__ wox, const float* __restrict__ woy,
    const float* __restrict__ woz, const float* __restrict__ ax, const float* __restrict__ ay,
    const float* __restrict__ f0p, const int64_t* __restrict__ nsamp,
    const int32_t* __restrict__ chunk_job, const int64_t* __restrict__ chunk_pbeg,
    const int64_t* __restrict__ chunk_pend, uint32_t k0, uint32_t k1,
    float* __restrict__ partial, uint64_t* __restrict__ rec) {
    const int32_t j = chunk_job[ch];
    const CellConst c = cell_setup(wox[j], woy[j], woz[j], ax[j], ay[j]);
    const float f0 = f0p ? f0p[j] : 1.0f;
    const uint64_t n = (uint64_t)nsamp[j];
    const uint64_t pbeg = (uint64_t)chunk_pbeg[ch];
    const uint64_t pend = (uint64_t)chunk_pend[ch];
    if (GRAD) {
        Comp out[4] = {Comp{0.0f, 0.0f}, Comp{0.0f, 0.0f}, Comp{0.0f, 0.0f}, Comp{0.0f, 0.0f}};
        float margin = -1.0f;
        if (c.ok) pairs_adj<64>(c, f0, pbeg, pend, n, (uint32_t)j, k0, k1, out, margin, lane);
#pragma unroll
        for (int a = 0; a < 4; ++a) out[a] = wave_reduce(out[a]);
        if (lane == 0) {
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                partial[(int64_t)ch * 8 + 2 * a] = out[a].s;
                partial[(int64_t)ch * 8 + 2 * a + 1] = out[a].c;
            }
        }
        store_flags_wave(margin, lane, rec + ch);
    } else {
        Comp acc[2] = {Comp{0.0f, 0.0f}, Comp{0.0f, 0.0f}};
        if (c.ok) pairs_fwd<64>(c, pbeg, pend, n, (uint32_t)j, k0, k1, acc, lane);
        const float a1 = acc[0].s + acc[0].c, a5 = acc[1].s + acc[1].c;
        Comp w = wave_reduce(Comp{__builtin_fmaf(f0, a1, (1.0f - f0) * a5), 0.0f});
        if (lane == 0) {
            partial[(int64_t)ch * 2] = w.s;
            partial[(int64_t)ch * 2 + 1] = w.c;
        }
    }
}

#define CAPVNDF_BATCH_PARAMS                                                                     \
    const float *__restrict__ wox, const float *__restrict__ woy, const float *__restrict__ woz, \
        const float *__restrict__ ax, const float *__restrict__ ay,                              \
        const float *__restrict__ f0p, const int64_t *__restrict__ nsamp,                        \
        const int32_t *__restrict__ chunk_job, const int64_t *__restrict__ chunk_pbeg,           \
        const int64_t *__restrict__ chunk_pend, const int32_t *__restrict__ owner_chunks,        \
        int32_t *__restrict__ counter, int32_t nchunks, uint32_t k0, uint32_t k1,              \
        float *__restrict__ partial, uint64_t *__restrict__ rec
#define CAPVNDF_CHUNK_ARGS wox, woy, woz, ax, ay, f0p, nsamp, chunk_job, chunk_pbeg, chunk_pend, \
                           k0, k1, partial, rec

// A block owns a chunk (block-wide reduction through LDS).
template <int BLOCK, bool GRAD, bool DYN>
__global__ __launch_bounds__(BLOCK) CAPVNDF_ADJ_ATTR void k_batch(CAPVNDF_BATCH_PARAMS) {
    // Loop control is made wave-uniform (readfirstlane) so that the compiler
    // emits scalar loops: the chunk loop contains barriers and cross-lane
    // reductions, which must not sit in a loop it treats as divergent.
    if (!DYN) {
        const int32_t cb = __builtin_amdgcn_readfirstlane(owner_chunks[blockIdx.x]);
        const int32_t ce = __builtin_amdgcn_readfirstlane(owner_chunks[blockIdx.x + 1]);
        for (int32_t ch = cb; ch < ce; ++ch) batch_chunk_block<BLOCK, GRAD>(ch, CAPVNDF_CHUNK_ARGS);
    } else {
        // At most nchunks + 1 tickets per owner: the loop ends even if a
        // miscompiled ticket read kept returning one chunk (that would leave
        // other slots unwritten, which the parity tests catch).
        __shared__ int32_t next;
        for (int32_t t = 0; t <= nchunks; ++t) {
            if (threadIdx.x == 0) next = atomicAdd(counter, 1);
            __syncthreads();
            const int32_t ch = __builtin_amdgcn_readfirstlane(next);
            __syncthreads();  // all have read `next` before thread 0 takes another
            if (ch >= nchunks) break;
            batch_chunk_block<BLOCK, GRAD>(ch, CAPVNDF_CHUNK_ARGS);
        }
    }
}

// A wavefront owns a chunk (smaller chunks, wave-only reduction, no LDS or
// barrier), so short jobs occupy 64 lanes instead of a whole block.
template <int BLOCK, bool GRAD, bool DYN>
__global__ __launch_bounds__(BLOCK) CAPVNDF_ADJ_ATTR void k_batch_wave(CAPVNDF_BATCH_PARAMS) {
    const uint32_t lane = threadIdx.x & 63;
    if (!DYN) {
        const int32_t wave =
            __builtin_amdgcn_readfirstlane((int32_t)(blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6)));
        const int32_t cb = __builtin_amdgcn_readfirstlane(owner_chunks[wave]);
        const int32_t ce = __builtin_amdgcn_readfirstlane(owner_chunks[wave + 1]);
        for (int32_t ch = cb; ch < ce; ++ch) batch_chunk_wave<GRAD>(ch, lane, CAPVNDF_CHUNK_ARGS);
    } else {
        // Every lane takes part in the atomic (lane 0 adds 1, the others 0)
        // and the ticket is read from lane 0 with readfirstlane, so the loop
        // has no lane-0 branch and its exit is a scalar branch.  With the add
        // under `if (lane == 0)` the compiler joined it to the lane-0 store
        // that ends the previous chunk and split the loop in two: lane 0 went
        // back to take a ticket while lanes 1-63 looped on with a zero ticket
        // and never left.  The ticket count is capped at nchunks + 1 as in
        // k_batch, so such a fault would give a wrong result, not a hang.
        for (int32_t t = 0; t <= nchunks; ++t) {
            const int32_t mine = atomicAdd(counter, lane == 0 ? 1 : 0);
            const int32_t ch = __builtin_amdgcn_readfirstlane(mine);
            if (ch >= nchunks) break;
            batch_chunk_wave<GRAD>(ch, lane, CAPVNDF_CHUNK_ARGS);
        }
    }
}
#undef CAPVNDF_CHUNK_ARGS
#undef CAPVNDF_BATCH_PARAMS

// Resets the dynamic scheduler's counter (a kernel, so that a captured graph
// holds no memset node).
__global__ void k_reset_counter(int32_t* counter) {
    if (threadIdx.x == 0) counter[0] = 0;
}

// ---------------------------------------------------------------------------
// Horizon fix pass: runs between an adjoint kernel and the finishing pass.
// An owner (a table block: cell, slot; or a batch chunk) has `threads`
// threads and a record of threads / 64 words, bit t set when thread t met a
// sample with margin >= 0.  For each such sample of a flagged thread's pairs
// the pass adds t64 - t32 (albedo_adj_f64 minus albedo_adj), the ws adjoint
// chained as the sample loops do, and merges the sums into the owner's
// partial in a fixed order: (A, gax, gay, gth) at partial[8 o ..] if
// WITH_VALUE, the three gradient sums at partial[6 o ..] otherwise.
//
// A wavefront reads its owners' records at once and returns if nothing was
// flagged.  Else it spreads flagged threads' pairs over its lanes and
// computes only their samples' margins (the forward sweep up to the
// reflection), two pairs per lane from two flagged threads, so that each
// lane runs two independent chains (one chain per lane left the scan bound
// by latency at about three wavefronts per SIMD).  The flagged samples go
// to a queue in LDS, which is evaluated one sample per lane: a chunk with
// hundreds of flagged samples costs a few double evaluations per wavefront,
// not hundreds.
//
// One wavefront per block: the block scheduler deals consecutive blocks to
// the 8 XCDs in turn, so the groups of one cell (or neighbouring chunks of
// one job) spread over all of them; with 4-wavefront blocks a cell's groups
// shared an XCD and the XCDs holding the smoothest, most grazing cells ran
// about twice as long as the others.
// ---------------------------------------------------------------------------
constexpr int kFixBlock = 64;

template <bool WITH_VALUE>
__device__ __forceinline__ void merge_fix(const Comp (&fix)[4], float* __restrict__ partial,
                                          int64_t o) {
    constexpr int A0 = WITH_VALUE ? 0 : 1;
    float* dst = partial + o * (WITH_VALUE ? 8 : 6);
#pragma unroll
    for (int a = A0; a < 4; ++a) {
        const Comp r = comp_merge(Comp{dst[2 * (a - A0)], dst[2 * (a - A0) + 1]}, fix[a]);
        dst[2 * (a - A0)] = r.s;
        dst[2 * (a - A0) + 1] = r.c;
    }
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask, uint32_t lane) {
    return (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
}

// Orders one wavefront's LDS accesses across its lanes (the writes before
// it are seen by the reads after it).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int32_t src) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src, 64);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src, 64);
    return ((uint64_t)hi << 32) | lo;
}

// The margins of pair p's two samples, the same arithmetic as the sample
// loops; -1 for a pair outside the owner (valid false) and for a second
// sample past the count n.  No branch: the two chains of a scan step stay
// in one basic block.
__device__ __forceinline__ void pair_margins(const CellConst& c, uint64_t p, bool valid,
                                             uint64_t n, uint32_t unit, uint32_t k0,
                                             uint32_t k1, float& m0, float& m1) {
    const Words ww = philox_pair(p, unit, kTagAlbedo, k0, k1);
    const float a = reflect_sample(c, unit24(ww.w0), unit24(ww.w1)).margin;
    const float b = reflect_sample(c, unit24(ww.w2), unit24(ww.w3)).margin;
    m0 = valid ? a : -1.0f;
    m1 = valid && 2 * p + 1 < n ? b : -1.0f;
}

// t64 - t32 of one flagged sample (code 2 p + h: pair p, its second sample
// when h = 1) as (A, gax, gay, gth), the ws adjoint chained.
__device__ __forceinline__ void sample_fix(const CellConst& c, float f0, uint64_t code,
                                           uint32_t unit, uint32_t k0, uint32_t k1,
                                           float (&v)[4]) {
    const Words ww = philox_pair(code >> 1, unit, kTagAlbedo, k0, k1);
    const bool second = (code & 1ull) != 0;
    const float u1 = unit24(second ? ww.w2 : ww.w0);
    const float u2 = unit24(second ? ww.w3 : ww.w1);
    const AdjTerm t = albedo_adj(c, f0, u1, u2);
    const AdjTerm d = albedo_adj_f64(c, f0, u1, u2);
    v[0] = d.w - t.w;
    v[1] = d.dax - t.dax;
    v[2] = d.day - t.day;
    v[3] = d.dth - t.dth;
    ws_chain(c, d.dwsx - t.dwsx, d.dwsy - t.dwsy, d.dzs - t.dzs, v[1], v[2], v[3]);
}

// The batch's fix pass: wavefront o serves chunk o (job chunk_job[o], pairs
// [chunk_pbeg[o], chunk_pend[o]), unit = job), whose thread t took the pairs
// pbeg + t + s * threads.  Lane k < threads / 64 loads record word k; the
// flagged threads are taken two at a time in thread order, lane l scanning
// pair s = s0 + l of both.  Each lane adds its samples' fixes to compensated
// sums, which are reduced in a fixed tree and merged into the chunk's
// partial (value and gradients).
constexpr int kFixQueue = 64;

__global__ __launch_bounds__(kFixBlock) void k_horizon_fix_batch(
    int64_t nchunks, int32_t threads, const float* __restrict__ wox,
    const float* __restrict__ woy, const float* __restrict__ woz, const float* __restrict__ ax,
    const float* __restrict__ ay, const float* __restrict__ f0p,
    const int64_t* __restrict__ nsamp, const int32_t* __restrict__ chunk_job,
    const int64_t* __restrict__ chunk_pbeg, const int64_t* __restrict__ chunk_pend, uint32_t k0,
    uint32_t k1, const uint64_t* __restrict__ rec, float* __restrict__ partial) {
    // the code (2 p + h) of each flagged sample found, in scan order
    __shared__ uint64_t queue[kFixQueue];
    const uint32_t lane = threadIdx.x & 63;
    const int64_t o = blockIdx.x;
    if (o >= nchunks) return;
    const int32_t nwords = threads >> 6;
    const uint64_t wd = (int32_t)lane < nwords ? rec[o * nwords + lane] : 0ull;
    uint64_t words = __ballot(wd != 0);
    if (words == 0) return;  // most chunks
    const int32_t u = chunk_job[o];
    const CellConst c = cell_setup(wox[u], woy[u], woz[u], ax[u], ay[u]);
    if (!c.ok) return;  // no samples were taken
    const float f0 = f0p ? f0p[u] : 1.0f;
    const uint64_t n = (uint64_t)nsamp[u];
    const uint64_t pbeg = (uint64_t)chunk_pbeg[o], pend = (uint64_t)chunk_pend[o];
    const uint32_t unit = (uint32_t)u;
    Comp corr[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) corr[a] = Comp{0.0f, 0.0f};
    uint32_t qn = 0;  // queued samples, the same in every lane

    auto flush = [&]() {
        wave_sync();
        if (lane < qn) {
            float v[4];
            sample_fix(c, f0, queue[lane], unit, k0, k1, v);
#pragma unroll
            for (int a = 0; a < 4; ++a) comp_add(corr[a], v[a]);
        }
        wave_sync();
        qn = 0;
    };
    // queues the lanes whose sample has margin >= 0
    auto note = [&](float margin, uint64_t code) {
        const uint64_t b = __ballot(margin >= 0.0f);
        const uint32_t nb = (uint32_t)__popcll(b);
        if (nb == 0) return;
        if (qn + nb > (uint32_t)kFixQueue) flush();
        if (margin >= 0.0f) queue[qn + lanes_below(b, lane)] = code;
        qn += nb;
    };
    // next flagged thread in thread order; false when none is left
    uint64_t m = 0;
    int32_t wi = 0;
    auto next = [&](uint32_t& t) -> bool {
        while (m == 0) {
            if (words == 0) return false;
            wi = __builtin_ctzll(words);
            words &= words - 1;
            m = shfl64(wd, wi);
        }
        t = (uint32_t)wi * 64 + (uint32_t)__builtin_ctzll(m);
        m &= m - 1;
        return true;
    };

    uint32_t ta, tb;
    while (next(ta)) {
        const bool two = next(tb);
        if (!two) tb = ta;
        // ta < tb: thread ta has at least as many pairs as tb
        for (uint64_t s0 = 0; pbeg + ta + s0 * (uint64_t)threads < pend; s0 += 64) {
            const uint64_t pa = pbeg + ta + (s0 + lane) * (uint64_t)threads;
            const uint64_t pb = pbeg + tb + (s0 + lane) * (uint64_t)threads;
            float a0, a1, b0, b1;
            pair_margins(c, pa, pa < pend, n, unit, k0, k1, a0, a1);
            pair_margins(c, pb, two && pb < pend, n, unit, k0, k1, b0, b1);
            note(a0, pa << 1);
            note(a1, (pa << 1) | 1ull);
            note(b0, pb << 1);
            note(b1, (pb << 1) | 1ull);
        }
    }
    if (qn != 0) flush();
#pragma unroll
    for (int a = 0; a < 4; ++a) corr[a] = wave_reduce(corr[a]);
    if (lane == 0) merge_fix<true>(corr, partial, o);
}

// The table's fix pass.  Wavefront w serves a group of kFixGroup owners of
// one cell (cell u = w / groups, slots g * kFixGroup + j, groups =
// ceil(slots / kFixGroup)); they share the cell's constants and Philox
// unit.  Lane l < 4 kFixGroup loads word l % 4 of owner l / 4 (one
// coalesced read), so a ballot of the nonzero words lists the flagged
// threads in owner order.  A thread holds kLutPairsPerThread = 32 pairs of
// each chunk, so a scan step gives one flagged thread half a wavefront and
// takes four (two per lane) when each slot holds one chunk; a slot of
// several chunks is scanned chunk by chunk, one thread per half wavefront,
// and a second owner joins only when it has one chunk.  The flagged samples
// are queued with their slot in owner order, so that each owner's entries
// are contiguous.  A queue of up to 2 x 64 samples is evaluated one sample
// per lane per round, each fix placed in LDS, and the lane that holds the
// first entry of an owner's run sums the run in queue order and merges it
// into that owner's partial (an owner whose run spans two queues is merged
// twice, in queue order).  Four owners per wavefront measured best with 32
// slots per cell (two chunks each): a cell holds up to about 500 flagged
// samples (grazing views of smooth surfaces, 2^20 samples), so more owners
// per wavefront leave a long tail (with 64 slots of one chunk, 16 owners
// took 1.4 times as long as 8), and fewer repeat the set-up more often.
constexpr int kFixGroup = 4;
constexpr int kFixTableQueue = 128;
static_assert(kLutPairsPerThread == 32, "a scan step gives each flagged thread 32 lanes");
static_assert(kFixGroup * (kLutBlock / 64) <= 64, "a group's records fit one wavefront");

template <bool WITH_VALUE>
__global__ __launch_bounds__(kFixBlock) void k_horizon_fix_table(
    int64_t ncells, const float* __restrict__ wox, const float* __restrict__ woy,
    const float* __restrict__ woz, const float* __restrict__ ax, const float* __restrict__ ay,
    const float* __restrict__ f0p, const int64_t* __restrict__ nsamp, int32_t slots,
    uint32_t unit_base, uint32_t k0, uint32_t k1, const uint64_t* __restrict__ rec,
    float* __restrict__ partial) {
    constexpr int nwords = kLutBlock / 64;
    __shared__ uint64_t q[kFixTableQueue];
    __shared__ int32_t qs[kFixTableQueue];
    __shared__ float qf[4][kFixTableQueue];
    const uint32_t lane = threadIdx.x & 63;
    const int64_t groups = (slots + kFixGroup - 1) / kFixGroup;
    const int64_t w = blockIdx.x;
    if (w >= ncells * groups) return;
    const int64_t u = w / groups;
    const int32_t s0 = (int32_t)(w - u * groups) * kFixGroup;
    const uint64_t n = (uint64_t)nsamp[u];
    const int64_t nch = cell_chunks((int64_t)n);
    const int64_t live = std::min<int64_t>(slots, nch);
    const int32_t my_slot = s0 + (int32_t)(lane / nwords);
    const uint64_t wd = lane < kFixGroup * nwords && my_slot < live
                            ? rec[(u * slots + my_slot) * nwords + lane % nwords]
                            : 0ull;
    uint64_t words = __ballot(wd != 0);
    if (words == 0) return;
    const CellConst c = cell_setup(wox[u], woy[u], woz[u], ax[u], ay[u]);
    if (!c.ok) return;  // no samples were taken
    const float f0 = f0p ? f0p[u] : 1.0f;
    const uint32_t unit = unit_base + (uint32_t)u;
    const uint64_t npairs = (n + 1) / 2;
    uint32_t qn = 0;  // the same in every lane

    auto flush = [&]() {
        wave_sync();
        for (uint32_t base = 0; base < qn; base += 64) {
            const uint32_t i = base + lane;
            float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            if (i < qn) sample_fix(c, f0, q[i], unit, k0, k1, v);
#pragma unroll
            for (int a = 0; a < 4; ++a) qf[a][i] = v[a];
        }
        wave_sync();
        for (uint32_t i = lane; i < qn; i += 64) {
            const int32_t s = qs[i];
            if (i != 0 && qs[i - 1] == s) continue;  // not the head of its run
            Comp f[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) f[a] = Comp{0.0f, 0.0f};
            for (uint32_t j = i; j < qn && qs[j] == s; ++j) {
#pragma unroll
                for (int a = 0; a < 4; ++a) comp_add(f[a], qf[a][j]);
            }
            merge_fix<WITH_VALUE>(f, partial, u * slots + s);
        }
        // an owner merged here may be merged again by another lane after a
        // later round: a workgroup barrier (the block is this wavefront)
        // orders those global accesses, and the LDS ones
        __syncthreads();
        qn = 0;
    };
    // queues the lane's flagged samples of pair p (slot s) in lane order
    auto push = [&](float m0, float m1, uint64_t p, int32_t s) {
        const bool g0 = m0 >= 0.0f, g1 = m1 >= 0.0f;
        const uint64_t b0 = __ballot(g0), b1 = __ballot(g1);
        const uint32_t nb = (uint32_t)(__popcll(b0) + __popcll(b1));
        if (nb == 0) return;
        if (qn + nb > (uint32_t)kFixTableQueue) flush();
        const uint32_t at = qn + lanes_below(b0, lane) + lanes_below(b1, lane);
        if (g0) {
            q[at] = p << 1;
            qs[at] = s;
        }
        if (g1) {
            q[at + (g0 ? 1 : 0)] = (p << 1) | 1ull;
            qs[at + (g0 ? 1 : 0)] = s;
        }
        qn += nb;
    };
    // next flagged (slot, thread) of the group in owner order; false when none
    uint64_t m = 0;
    int32_t wi = 0;
    auto next = [&](int32_t& s, uint32_t& t) -> bool {
        while (m == 0) {
            if (words == 0) return false;
            wi = __builtin_ctzll(words);
            words &= words - 1;
            m = shfl64(wd, wi);
        }
        s = s0 + wi / nwords;
        t = (uint32_t)(wi % nwords) * 64 + (uint32_t)__builtin_ctzll(m);
        m &= m - 1;
        return true;
    };
    // lane k of a half wavefront takes pair k of its thread's chunk ch
    const uint32_t half = lane >> 5, k = lane & 31;
    auto chunk_pair = [&](int64_t ch, uint32_t t, bool& valid) -> uint64_t {
        const uint64_t b = (uint64_t)ch * kLutChunkPairs;
        const uint64_t p = b + t + (uint64_t)k * kLutBlock;
        valid = valid && p < std::min(b + kLutChunkPairs, npairs);
        return p;
    };

    int32_t sa, sb;
    uint32_t ta, tb;
    bool more = next(sa, ta);
    while (more) {
        // chunks s, s + slots, ... of the cell belong to slot s; the count
        // does not grow with s, so once it is 1 it stays 1
        const int64_t rounds = (nch - sa + slots - 1) / slots;
        if (rounds == 1) {
            // up to four threads: lanes 0-31 take the first and third,
            // lanes 32-63 the second and fourth (queued in that order)
            int32_t s1 = sa, s2 = sa, s3 = sa;
            uint32_t t1 = ta, t2 = ta, t3 = ta;
            int32_t ni = 1;
            if (next(s1, t1)) {
                ni = 2;
                if (next(s2, t2)) {
                    ni = 3;
                    if (next(s3, t3)) ni = 4;
                }
            }
            const int32_t sx = half ? s1 : sa, sy = half ? s3 : s2;
            const uint32_t tx = half ? t1 : ta, ty = half ? t3 : t2;
            bool vx = half == 0 || ni >= 2, vy = half ? ni >= 4 : ni >= 3;
            const uint64_t px = chunk_pair(sx, tx, vx);
            const uint64_t py = chunk_pair(sy, ty, vy);
            float x0, x1, y0, y1;
            pair_margins(c, px, vx, n, unit, k0, k1, x0, x1);
            pair_margins(c, py, vy, n, unit, k0, k1, y0, y1);
            push(x0, x1, px, sx);
            push(y0, y1, py, sy);
            more = next(sa, ta);
            continue;
        }
        bool two = next(sb, tb);
        // a second owner joins only when it holds one chunk, else its
        // entries would interleave with the first's
        const bool carry = two && sb != sa;
        if (carry) two = false;
        const int32_t s = half && two ? sb : sa;
        const uint32_t t = half && two ? tb : ta;
        for (int64_t r = 0; r < rounds; ++r) {
            const int64_t ch = s + r * slots;
            bool v = (half == 0 || two) && ch < nch;
            const uint64_t p = chunk_pair(ch, t, v);
            float m0, m1;
            pair_margins(c, p, v, n, unit, k0, k1, m0, m1);
            push(m0, m1, p, s);
        }
        if (carry) {
            sa = sb;
            ta = tb;
        } else {
            more = next(sa, ta);
        }
    }
    if (qn != 0) flush();
}

// The batch fix pass over a plan's nchunks chunks of `threads` threads.
void launch_fix_batch(int64_t nchunks, int32_t threads, const float* wox, const float* woy,
                      const float* woz, const float* ax, const float* ay, const float* f0,
                      const int64_t* nsamp, const int32_t* chunk_job, const int64_t* chunk_pbeg,
                      const int64_t* chunk_pend, uint32_t k0, uint32_t k1, const uint64_t* rec,
                      float* part, hipStream_t st) {
    hipLaunchKernelGGL(k_horizon_fix_batch, dim3((unsigned)nchunks), dim3(kFixBlock), 0, st,
                       nchunks, threads, wox, woy, woz, ax, ay, f0, nsamp, chunk_job, chunk_pbeg,
                       chunk_pend, k0, k1, rec, part);
}

// ---------------------------------------------------------------------------
// Finishing pass: unit u merges its partials in order, divides by its sample
// count and applies an optional per-unit scale.  Partials of unit u: the
// first min(slots, chunks) of [u * slots, (u + 1) * slots) if unit_chunks is
// NULL (table estimators), else [unit_chunks[u], unit_chunks[u + 1]) (batch
// plans).  A count outside [0, 2^40) gives NaN.
// ---------------------------------------------------------------------------
template <int NACC>
__global__ __launch_bounds__(kFinishBlock) void k_finish(
    int64_t nunits, const float* __restrict__ partial, int32_t slots,
    const int32_t* __restrict__ unit_chunks, const int64_t* __restrict__ nsamp,
    const float* __restrict__ scale, float* __restrict__ o0, float* __restrict__ o1,
    float* __restrict__ o2, float* __restrict__ o3) {
    const int64_t u = (int64_t)blockIdx.x * kFinishBlock + threadIdx.x;
    if (u >= nunits) return;
    const int64_t n = nsamp[u];
    int64_t cb, ce;
    if (unit_chunks) {
        cb = unit_chunks[u];
        ce = unit_chunks[u + 1];
    } else {
        cb = u * slots;
        ce = cb + std::min<int64_t>(slots, cell_chunks(n));
    }
    Comp r[NACC];
#pragma unroll
    for (int a = 0; a < NACC; ++a) r[a] = Comp{0.0f, 0.0f};
    for (int64_t ch = cb; ch < ce; ++ch) {
#pragma unroll
        for (int a = 0; a < NACC; ++a) {
            const float* p = partial + (ch * NACC + a) * 2;
            r[a] = comp_merge(r[a], Comp{p[0], p[1]});
        }
    }
    const bool bad = n < 0 || n >= kMaxSamples;
    const float inv = n > 0 && !bad ? (float)(1.0 / (double)n) : 0.0f;
    const float sc = (scale ? scale[u] : 1.0f) * inv;
    float* outs[4] = {o0, o1, o2, o3};
#pragma unroll
    for (int a = 0; a < NACC; ++a) outs[a][u] = bad ? __builtin_nanf("") : (r[a].s + r[a].c) * sc;
}

inline unsigned finish_grid(int64_t n) { return (unsigned)((n + kFinishBlock - 1) / kFinishBlock); }

// Slots per cell.  A call aims for kFillBlocks blocks (about four rounds of
// the blocks the chip holds at once) with at least kMinSlots per cell, and
// stays below 2^24 blocks (a dispatch counts its work-items in 32 bits).
// On 4096 cells of 2^20 samples (64 chunks each) 32 slots measured faster
// than 64 (value + gradient 0.8 %, forward 1.3 %; the recompute-style
// backward 0.5 % slower) and than 16 (value + gradient 1.8 % slower).
constexpr int64_t kFillBlocks = 8192;
constexpr int64_t kMinSlots = 32;
constexpr int64_t kMaxBlocks = ((int64_t)1 << 24) - 1;

int64_t target_slots(int64_t ncells) {
    const int64_t s = std::max<int64_t>(kMinSlots, (kFillBlocks + ncells - 1) / ncells);
    return std::max<int64_t>(1, std::min<int64_t>(s, kMaxBlocks / ncells));
}

// Workspace of a table launch: the partials (slot-major, as k_finish reads
// them), then for the adjoint kernels the horizon records.
size_t table_bytes(int64_t ncells, int64_t slots, int nacc, bool records) {
    const int64_t nowners = ncells * slots;
    return (size_t)nowners * nacc * 2 * sizeof(float) +
           (records ? rec_bytes(nowners, kLutBlock / 64) : 0);
}

uint64_t* records_after(float* part, int64_t ncells, int32_t slots, int nacc) {
    return reinterpret_cast<uint64_t*>(part + (size_t)ncells * (size_t)slots * (size_t)(2 * nacc));
}

// The fix pass over a table launch of ncells cells and `slots` slots.
template <bool WITH_VALUE>
void launch_table_fix(int64_t ncells, int32_t slots, const float* wox, const float* woy,
                      const float* woz, const float* ax, const float* ay, const float* f0,
                      const int64_t* nsamples, uint32_t unit_base, uint32_t k0, uint32_t k1,
                      uint64_t* rec, float* part, hipStream_t st) {
    const int64_t waves = ncells * ((slots + kFixGroup - 1) / kFixGroup);
    hipLaunchKernelGGL(k_horizon_fix_table<WITH_VALUE>, dim3((unsigned)waves), dim3(kFixBlock), 0,
                       st, ncells, wox, woy, woz, ax, ay, f0, nsamples, slots, unit_base, k0, k1,
                       rec, part);
}

// Argument checks of the table estimators and the slot count the workspace
// allows: min(target_slots(ncells), workspace_bytes / (ncells * slot bytes)).
int32_t prepare_cells(const char* fn, int64_t ncells, const float* wox, const float* woy,
                      const float* woz, const float* ax, const float* ay, const int64_t* nsamples,
                      int nacc, bool records, const void* workspace, size_t workspace_bytes,
                      int32_t* slots) {
    *slots = 0;
    if (ncells < 0) return fail(CAPVNDF_ERR_BAD_SIZE, "%s: ncells < 0", fn);
    if (ncells > kMaxBlocks)
        return fail(CAPVNDF_ERR_BAD_SIZE, "%s: ncells must be below 2^24; split the cells over "
                    "several calls", fn);
    if (ncells == 0) return CAPVNDF_OK;
    const void* req[] = {wox, woy, woz, ax, ay};
    const char* names[] = {"wox", "woy", "woz", "ax", "ay"};
    for (int i = 0; i < 5; ++i)
        if (int32_t rc = check_array(req[i], names[i])) return rc;
    if (nsamples == nullptr) return fail(CAPVNDF_ERR_NULL_PTR, "%s: nsamples is NULL", fn);
    if (!aligned_to(nsamples, 8))
        return fail(CAPVNDF_ERR_MISALIGNED, "%s: nsamples must be 8-byte aligned", fn);
    const size_t least = table_bytes(ncells, 1, nacc, records);
    if (workspace == nullptr || workspace_bytes < least)
        return fail(CAPVNDF_ERR_WORKSPACE, "%s: workspace of at least %zu bytes needed, %zu given",
                    fn, least, workspace == nullptr ? (size_t)0 : workspace_bytes);
    if (!aligned_to(workspace, 16))
        return fail(CAPVNDF_ERR_MISALIGNED, "%s: workspace must be 16-byte aligned", fn);
    // table_bytes is affine in the slot count: fixed + slots * per_slot.
    // One-sum calls (the value-only pass, radiance) count slots at the
    // two-sum forward's size: albedo_workspace_size(.., 0) sizes for two sums
    // per slot, up to the largest cell's chunk count when given the host
    // counts, so the same workspace gives the three calls the same slots.  At
    // half the size per slot a one-sum call got twice as many, and a block
    // without a chunk costs about as much as one with a chunk when the
    // blocks each hold one (dispatch-bound: 2^18 samples per cell ran at
    // half the rate).
    const int sizing = nacc == 1 && !records ? 2 : nacc;
    const size_t fixed = table_bytes(ncells, 0, sizing, records);
    const size_t per_slot = table_bytes(ncells, 1, sizing, records) - fixed;
    *slots = (int32_t)std::min<int64_t>(
        target_slots(ncells),
        std::max<int64_t>(1, (int64_t)((workspace_bytes - fixed) / per_slot)));
    return CAPVNDF_OK;
}

}  // namespace
}  // namespace capvndf

using namespace capvndf;

extern "C" size_t albedo_workspace_size(int64_t ncells, const int64_t* nsamples_host,
                                        int32_t with_grad) {
    if (ncells <= 0 || ncells > kMaxBlocks || (with_grad != 0 && with_grad != 1)) return 0;
    int64_t slots = target_slots(ncells);
    if (nsamples_host != nullptr) {
        int64_t most = 0;
        for (int64_t c = 0; c < ncells; ++c) {
            const int64_t n = nsamples_host[c];
            if (n < 0 || n >= kMaxSamples) return 0;
            most = std::max(most, cell_chunks(n));
        }
        slots = std::min(slots, std::max<int64_t>(1, most));
    }
    return with_grad ? table_bytes(ncells, slots, 4, true) : table_bytes(ncells, slots, 2, false);
}

extern "C" int32_t albedo_estimate(int64_t ncells, const float* wox, const float* woy,
                                   const float* woz, const float* ax, const float* ay,
                                   const int64_t* nsamples, uint64_t seed, float* s_f1,
                                   float* s_f5, void* workspace, size_t workspace_bytes,
                                   void* stream) {
    int32_t slots = 0;
    if (int32_t rc = prepare_cells("albedo_estimate", ncells, wox, woy, woz, ax, ay, nsamples, 2,
                                   false, workspace, workspace_bytes, &slots))
        return rc;
    if (ncells == 0) return CAPVNDF_OK;
    if (int32_t rc = check_array(s_f1, "s_f1")) return rc;
    if (int32_t rc = check_array(s_f5, "s_f5")) return rc;
    const hipStream_t st = as_stream(stream);
    float* part = static_cast<float*>(workspace);
    hipLaunchKernelGGL(k_albedo_fwd<0>, dim3((unsigned)(ncells * slots)), dim3(kLutBlock), 0, st,
                       wox, woy, woz, ax, ay, nullptr, nsamples, slots, 0u, key_lo(seed),
                       key_hi(seed), part);
    if (int32_t rc = check_launch("albedo_estimate launch")) return rc;
    hipLaunchKernelGGL(k_finish<2>, dim3(finish_grid(ncells)), dim3(kFinishBlock), 0, st, ncells,
                       part, slots, nullptr, nsamples, nullptr, s_f1, s_f5, nullptr, nullptr);
    return check_launch("albedo_estimate finish launch");
}

extern "C" int32_t albedo_estimate_backward(int64_t ncells, const float* wox, const float* woy,
                                            const float* woz, const float* ax, const float* ay,
                                            const int64_t* nsamples, uint64_t seed,
                                            const float* f0, const float* grad_albedo,
                                            float* grad_ax, float* grad_ay, float* grad_theta_o,
                                            void* workspace, size_t workspace_bytes,
                                            void* stream) {
    int32_t slots = 0;
    if (int32_t rc = prepare_cells("albedo_estimate_backward", ncells, wox, woy, woz, ax, ay,
                                   nsamples, 3, true, workspace, workspace_bytes, &slots))
        return rc;
    if (ncells == 0) return CAPVNDF_OK;
    if (int32_t rc = check_array(grad_ax, "grad_ax")) return rc;
    if (int32_t rc = check_array(grad_ay, "grad_ay")) return rc;
    if (int32_t rc = check_array(grad_theta_o, "grad_theta_o")) return rc;
    if (f0 != nullptr)
        if (int32_t rc = check_array(f0, "f0")) return rc;
    if (grad_albedo != nullptr)
        if (int32_t rc = check_array(grad_albedo, "grad_albedo")) return rc;
    const hipStream_t st = as_stream(stream);
    float* part = static_cast<float*>(workspace);
    uint64_t* rec = records_after(part, ncells, slots, 3);
    hipLaunchKernelGGL(k_albedo_adj<false>, dim3((unsigned)(ncells * slots)), dim3(kLutBlock), 0,
                       st, wox, woy, woz, ax, ay, f0, nsamples, slots, 0u, key_lo(seed),
                       key_hi(seed), part, rec);
    if (int32_t rc = check_launch("albedo_estimate_backward launch")) return rc;
    launch_table_fix<false>(ncells, slots, wox, woy, woz, ax, ay, f0, nsamples, 0u, key_lo(seed),
                            key_hi(seed), rec, part, st);
    if (int32_t rc = check_launch("albedo_estimate_backward fix launch")) return rc;
    hipLaunchKernelGGL(k_finish<3>, dim3(finish_grid(ncells)), dim3(kFinishBlock), 0, st, ncells,
                       part, slots, nullptr, nsamples, grad_albedo, grad_ax, grad_ay, grad_theta_o,
                       nullptr);
    return check_launch("albedo_estimate_backward finish launch");
}

namespace capvndf {
namespace {

// albedo_value_and_grad on a given partial buffer with a given slot count
// (shared by the workspace entry point and its variant on the library's own
// buffer).
int32_t enqueue_value_and_grad(int64_t ncells, const float* wox, const float* woy,
                               const float* woz, const float* ax, const float* ay,
                               const int64_t* nsamples, uint64_t seed, const float* f0,
                               float* albedo, float* grad_ax, float* grad_ay, float* grad_theta_o,
                               bool grad, float* part, int32_t slots, hipStream_t st) {
    const dim3 grid((unsigned)(ncells * slots)), block(kLutBlock);
    if (grad) {
        uint64_t* rec = records_after(part, ncells, slots, 4);
        hipLaunchKernelGGL(k_albedo_adj<true>, grid, block, 0, st, wox, woy, woz, ax, ay, f0,
                           nsamples, slots, 0u, key_lo(seed), key_hi(seed), part, rec);
        if (int32_t rc = check_launch("albedo_value_and_grad launch")) return rc;
        launch_table_fix<true>(ncells, slots, wox, woy, woz, ax, ay, f0, nsamples, 0u,
                               key_lo(seed), key_hi(seed), rec, part, st);
        if (int32_t rc = check_launch("albedo_value_and_grad fix launch")) return rc;
        hipLaunchKernelGGL(k_finish<4>, dim3(finish_grid(ncells)), dim3(kFinishBlock), 0, st, ncells,
                           part, slots, nullptr, nsamples, nullptr, albedo, grad_ax, grad_ay,
                           grad_theta_o);
    } else {
        hipLaunchKernelGGL(k_albedo_fwd<1>, grid, block, 0, st, wox, woy, woz, ax, ay, f0,
                           nsamples, slots, 0u, key_lo(seed), key_hi(seed), part);
        if (int32_t rc = check_launch("albedo_value_and_grad launch")) return rc;
        hipLaunchKernelGGL(k_finish<1>, dim3(finish_grid(ncells)), dim3(kFinishBlock), 0, st, ncells,
                           part, slots, nullptr, nsamples, nullptr, albedo, nullptr, nullptr,
                           nullptr);
    }
    return check_launch("albedo_value_and_grad finish launch");
}

// Output checks of albedo_value_and_grad; *grad tells whether the three
// gradient outputs are given.
int32_t check_value_and_grad_outputs(const char* fn, const float* f0, const float* albedo,
                                     const float* grad_ax, const float* grad_ay,
                                     const float* grad_theta_o, bool* grad) {
    if (int32_t rc = check_array(albedo, "albedo")) return rc;
    const int ngrad = (grad_ax != nullptr) + (grad_ay != nullptr) + (grad_theta_o != nullptr);
    if (ngrad != 0 && ngrad != 3)
        return fail(CAPVNDF_ERR_NULL_PTR, "%s: give all three gradient outputs or none", fn);
    *grad = ngrad == 3;
    if (*grad) {
        if (int32_t rc = check_array(grad_ax, "grad_ax")) return rc;
        if (int32_t rc = check_array(grad_ay, "grad_ay")) return rc;
        if (int32_t rc = check_array(grad_theta_o, "grad_theta_o")) return rc;
    }
    if (f0 != nullptr)
        if (int32_t rc = check_array(f0, "f0")) return rc;
    return CAPVNDF_OK;
}

}  // namespace
}  // namespace capvndf

extern "C" int32_t albedo_value_and_grad(int64_t ncells, const float* wox, const float* woy,
                                         const float* woz, const float* ax, const float* ay,
                                         const int64_t* nsamples, uint64_t seed, const float* f0,
                                         float* albedo, float* grad_ax, float* grad_ay,
                                         float* grad_theta_o, void* workspace,
                                         size_t workspace_bytes, void* stream) {
    const char* fn = "albedo_value_and_grad";
    bool grad = false;
    if (ncells > 0)
        if (int32_t rc = check_value_and_grad_outputs(fn, f0, albedo, grad_ax, grad_ay,
                                                      grad_theta_o, &grad))
            return rc;
    int32_t slots = 0;
    if (int32_t rc = prepare_cells(fn, ncells, wox, woy, woz, ax, ay, nsamples, grad ? 4 : 1,
                                   grad, workspace, workspace_bytes, &slots))
        return rc;
    if (ncells == 0) return CAPVNDF_OK;
    return enqueue_value_and_grad(ncells, wox, woy, woz, ax, ay, nsamples, seed, f0, albedo,
                                  grad_ax, grad_ay, grad_theta_o, grad,
                                  static_cast<float*>(workspace), slots, as_stream(stream));
}

extern "C" int32_t radiance_estimate(int64_t ncells, const float* wox, const float* woy,
                                     const float* woz, const float* ax, const float* ay,
                                     const float* f0, const int64_t* nsamples, uint64_t seed,
                                     const float* lobes, int32_t nlobes, float* radiance,
                                     void* workspace, size_t workspace_bytes, void* stream) {
    if (nlobes < 0 || nlobes > kMaxLobes)
        return fail(CAPVNDF_ERR_BAD_SIZE, "radiance_estimate: nlobes must be in [0, %d]", kMaxLobes);
    int32_t slots = 0;
    if (int32_t rc = prepare_cells("radiance_estimate", ncells, wox, woy, woz, ax, ay, nsamples, 1,
                                   false, workspace, workspace_bytes, &slots))
        return rc;
    if (ncells == 0) return CAPVNDF_OK;
    if (int32_t rc = check_array(radiance, "radiance")) return rc;
    if (nlobes > 0)
        if (int32_t rc = check_array(lobes, "lobes")) return rc;
    if (f0 != nullptr)
        if (int32_t rc = check_array(f0, "f0")) return rc;
    const hipStream_t st = as_stream(stream);
    float* part = static_cast<float*>(workspace);
    const dim3 grid((unsigned)(ncells * slots)), block(kLutBlock);
    const uint32_t k0 = key_lo(seed), k1 = key_hi(seed);
    static_assert(kMaxLobes == 8, "the switch below covers 0 .. 8 lobes");
#define CAPVNDF_LAUNCH_RADIANCE(NL)                                                                \
    case NL:                                                                                       \
        hipLaunchKernelGGL(k_radiance<NL>, grid, block, 0, st, wox, woy, woz, ax, ay, f0, lobes,  \
                           nsamples, slots, k0, k1, part);                                         \
        break;
    switch (nlobes) {
        CAPVNDF_LAUNCH_RADIANCE(0)
        CAPVNDF_LAUNCH_RADIANCE(1)
        CAPVNDF_LAUNCH_RADIANCE(2)
        CAPVNDF_LAUNCH_RADIANCE(3)
        CAPVNDF_LAUNCH_RADIANCE(4)
        CAPVNDF_LAUNCH_RADIANCE(5)
        CAPVNDF_LAUNCH_RADIANCE(6)
        CAPVNDF_LAUNCH_RADIANCE(7)
        CAPVNDF_LAUNCH_RADIANCE(8)
        default:
            return fail(CAPVNDF_ERR_BAD_SIZE, "radiance_estimate: nlobes must be in [0, %d]", kMaxLobes);
    }
#undef CAPVNDF_LAUNCH_RADIANCE
    if (int32_t rc = check_launch("radiance_estimate launch")) return rc;
    hipLaunchKernelGGL(k_finish<1>, dim3(finish_grid(ncells)), dim3(kFinishBlock), 0, st, ncells,
                       part, slots, nullptr, nsamples, nullptr, radiance, nullptr, nullptr,
                       nullptr);
    return check_launch("radiance_estimate finish launch");
}

// ===========================================================================
// albedo_value_and_grad on a partial buffer the library owns, for callers
// that cannot allocate device memory.  The buffer is a file-scope device
// array; host code never passes its name to a kernel, only the device
// address hipGetSymbolAddress returns for the current device (each device
// holds its own copy), taken once per device on the first call there.
// Nothing in it needs clearing: every partial and horizon record a call
// reads was written by the same call.  Calls that overlap on one device race
// on it.
// ===========================================================================
namespace capvndf {
namespace {

constexpr size_t kScratchBytes = (size_t)16 << 20;
__device__ __align__(256) float scratch[kScratchBytes / sizeof(float)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
float* g_scratch[kMaxDevices] = {};

int32_t scratch_of_current_device(const char* fn, float** out) {
    int dev = 0;
    if (int32_t rc = check_hip(hipGetDevice(&dev), "hipGetDevice")) return rc;
    if (dev < 0 || dev >= kMaxDevices)
        return fail(CAPVNDF_ERR_BAD_ARG, "%s: device %d beyond the %d this library tracks", fn, dev,
                    kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch[dev] == nullptr) {
        void* ptr = nullptr;
        if (int32_t rc = check_hip(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)),
                                   "hipGetSymbolAddress (scratch)"))
            return rc;
        g_scratch[dev] = static_cast<float*>(ptr);
    }
    *out = g_scratch[dev];
    return CAPVNDF_OK;
}

}  // namespace
}  // namespace capvndf

extern "C" int32_t albedo_value_and_grad_noalloc(int64_t ncells, const float* wox,
                                                 const float* woy, const float* woz,
                                                 const float* ax, const float* ay,
                                                 const int64_t* nsamples, uint64_t seed,
                                                 const float* f0, float* albedo, float* grad_ax,
                                                 float* grad_ay, float* grad_theta_o,
                                                 void* stream) {
    const char* fn = "albedo_value_and_grad_noalloc";
    bool grad = false;
    if (ncells > 0)
        if (int32_t rc = check_value_and_grad_outputs(fn, f0, albedo, grad_ax, grad_ay,
                                                      grad_theta_o, &grad))
            return rc;
    // one slot per cell: partials, and with gradients the horizon record
    const size_t per_cell = table_bytes(1, 1, grad ? 4 : 1, grad);
    if (ncells > (int64_t)(kScratchBytes / per_cell))
        return fail(CAPVNDF_ERR_BAD_SIZE,
                    "%s: at most %lld cells per call %s gradients (the library's buffer holds "
                    "%zu bytes); use albedo_value_and_grad with a workspace", fn,
                    (long long)(kScratchBytes / per_cell), grad ? "with" : "without",
                    kScratchBytes);
    if (ncells <= 0) {
        int32_t slots = 0;
        return prepare_cells(fn, ncells, wox, woy, woz, ax, ay, nsamples, 1, false, nullptr, 0,
                             &slots);
    }
    float* buf = nullptr;
    if (int32_t rc = scratch_of_current_device(fn, &buf)) return rc;
    int32_t slots = 0;
    if (int32_t rc = prepare_cells(fn, ncells, wox, woy, woz, ax, ay, nsamples, grad ? 4 : 1,
                                   grad, buf, kScratchBytes, &slots))
        return rc;
    return enqueue_value_and_grad(ncells, wox, woy, woz, ax, ay, nsamples, seed, f0, albedo,
                                  grad_ax, grad_ay, grad_theta_o, grad, buf, slots,
                                  as_stream(stream));
}


// ===========================================================================
// Register-resident estimator microbenchmark: each lane runs the per-sample
// arithmetic of one estimator kernel over `pairs` Philox pairs of its own
// stream (tag 3, unit = lane) into plain per-lane sums -- no loads in the
// loop, no compensated sums, no cross-lane reductions -- at the estimator
// kernel's own occupancy.  KIND 0: the forward's two sums; 1: value and
// adjoint; 2: direct illumination under 4 lobes.  Its issue rate is what the
// estimator's instruction mix reaches on this chip with nothing else in the
// way, the ceiling the table kernels are measured against.
// ===========================================================================
namespace capvndf {
namespace {

template <int KIND>
__device__ __forceinline__ float microbench_lane(int64_t t, int32_t pairs, uint32_t k0,
                                                 uint32_t k1, const Lobes<4>& lobes) {
    // the lane's cell: view uniform over the hemisphere, alpha = 10^(-2 U)
    const Words w = philox_pair(0, (uint32_t)t, 6u, k0, k1);
    const float mu = 1.0f - unit24(w.w0);
    float sp, cp;
    sincos_turns(unit24(w.w1), &sp, &cp);
    const float sz = fsqrt(fmaxf(__builtin_fmaf(-mu, mu, 1.0f), 0.0f));
    const float ax = __builtin_amdgcn_exp2f(-6.643856189774724f * unit24(w.w2));
    const float ay = __builtin_amdgcn_exp2f(-6.643856189774724f * unit24(w.w3));
    const CellConst c = cell_setup(sz * cp, sz * sp, mu, ax, ay);
    float acc[7] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    float mf = -1.0f;
    for (int32_t p = 0; p < pairs; ++p) {
        const Words q = philox_pair((uint64_t)p, (uint32_t)t, kTagAlbedo, k0, k1);
        const float u[4] = {unit24(q.w0), unit24(q.w1), unit24(q.w2), unit24(q.w3)};
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            if (KIND == 0) {
                const FwdTerm r = albedo_fwd(c, u[2 * j], u[2 * j + 1]);
                acc[0] += r.g;
                acc[1] = __builtin_fmaf(r.g, r.m5, acc[1]);
            } else if (KIND == 1) {
                const AdjTerm r = albedo_adj(c, 0.04f, u[2 * j], u[2 * j + 1]);
                acc[0] += r.w; acc[1] += r.dax; acc[2] += r.day; acc[3] += r.dth;
                acc[4] += r.dwsx; acc[5] += r.dwsy; acc[6] += r.dzs;
                mf = fmaxf(mf, r.margin);  // the loops' flag
            } else {
                acc[0] += radiance_term(c, 0.04f, lobes, u[2 * j], u[2 * j + 1]);
            }
        }
    }
    return ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + acc[6]) +
           mf;
}

template <int KIND>
__global__ __launch_bounds__(kLutBlock) void k_estimator_microbench(
    int64_t lanes, int32_t pairs, uint32_t k0, uint32_t k1, const float* __restrict__ lobep,
    uint32_t* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * kLutBlock + threadIdx.x;
    if (t >= lanes) return;
    const Lobes<4> lobes = KIND == 2 ? load_lobes<4>(lobep) : Lobes<4>{};
    out[t] = __float_as_uint(microbench_lane<KIND>(t, pairs, k0, k1, lobes));
}

template <>
__global__ __launch_bounds__(kLutBlock) CAPVNDF_ADJ_ATTR void k_estimator_microbench<1>(
    int64_t lanes, int32_t pairs, uint32_t k0, uint32_t k1, const float* __restrict__ lobep,
    uint32_t* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * kLutBlock + threadIdx.x;
    if (t >= lanes) return;
    (void)lobep;
    out[t] = __float_as_uint(microbench_lane<1>(t, pairs, k0, k1, Lobes<4>{}));
}

}  // namespace
}  // namespace capvndf

extern "C" int32_t estimator_microbench(int32_t kind, int64_t lanes, int32_t pairs, uint64_t seed,
                                        const float* lobes, uint32_t* out, void* stream) {
    if (lanes < 0 || lanes > ((int64_t)1 << 31) || pairs < 0)
        return fail(CAPVNDF_ERR_BAD_SIZE,
                    "estimator_microbench: lanes must be in [0, 2^31], pairs >= 0");
    if (kind < 0 || kind > 2)
        return fail(CAPVNDF_ERR_BAD_ARG, "estimator_microbench: kind must be 0, 1 or 2");
    if (lanes == 0) return CAPVNDF_OK;
    if (int32_t rc = check_array(out, "out")) return rc;
    if (kind == 2)
        if (int32_t rc = check_array(lobes, "lobes")) return rc;
    const dim3 grid((unsigned)((lanes + kLutBlock - 1) / kLutBlock)), block(kLutBlock);
    const hipStream_t st = as_stream(stream);
    const uint32_t k0 = key_lo(seed), k1 = key_hi(seed);
    if (kind == 0)
        hipLaunchKernelGGL(k_estimator_microbench<0>, grid, block, 0, st, lanes, pairs, k0, k1,
                           lobes, out);
    else if (kind == 1)
        hipLaunchKernelGGL(k_estimator_microbench<1>, grid, block, 0, st, lanes, pairs, k0, k1,
                           lobes, out);
    else
        hipLaunchKernelGGL(k_estimator_microbench<2>, grid, block, 0, st, lanes, pairs, k0, k1,
                           lobes, out);
    return check_launch("estimator_microbench launch");
}

// ===========================================================================
// Element-wise helpers of the differentiable albedo: the view direction from
// its spherical angles, and the chain rule through the diagonal Jacobian.
// ===========================================================================
namespace capvndf {
namespace {

constexpr int kEltBlock = 256;
constexpr int64_t kEltMaxBlocks = (int64_t)1 << 20;  // grid-stride beyond this

inline unsigned elt_grid(int64_t n) {
    const int64_t b = (n + kEltBlock - 1) / kEltBlock;
    return (unsigned)(b < kEltMaxBlocks ? b : kEltMaxBlocks);
}

// wo = (sin t cos p, sin t sin p, cos t), the parametrisation whose polar
// derivative the adjoint reports.
__global__ __launch_bounds__(kEltBlock) void k_view_from_angles(
    int64_t n, const float* __restrict__ theta, const float* __restrict__ phi,
    float* __restrict__ wox, float* __restrict__ woy, float* __restrict__ woz) {
    const int64_t stride = (int64_t)gridDim.x * kEltBlock;
    for (int64_t i = (int64_t)blockIdx.x * kEltBlock + threadIdx.x; i < n; i += stride) {
        float st, ct, sp, cp;
        sincosf(theta[i], &st, &ct);
        sincosf(phi[i], &sp, &cp);
        wox[i] = st * cp;
        woy[i] = st * sp;
        woz[i] = ct;
    }
}

// out_k = g * d_k for the three parameter derivatives that are given, and
// g * (s_f1 - s_f5) for F0 (the estimate is linear in F0).  Every input of an
// element is read before any output of it is written, so outputs may alias
// inputs (no __restrict__).
__global__ __launch_bounds__(kEltBlock) void k_apply_jacobian(
    int64_t n, const float* g, const float* dx, const float* dy, const float* dt,
    const float* s1, const float* s5, float* ox, float* oy, float* ot, float* of) {
    const int64_t stride = (int64_t)gridDim.x * kEltBlock;
    for (int64_t i = (int64_t)blockIdx.x * kEltBlock + threadIdx.x; i < n; i += stride) {
        const float gi = g[i];
        const float vx = dx ? dx[i] : 0.0f;
        const float vy = dy ? dy[i] : 0.0f;
        const float vt = dt ? dt[i] : 0.0f;
        const float vf = s1 ? s1[i] - s5[i] : 0.0f;
        if (dx) ox[i] = gi * vx;
        if (dy) oy[i] = gi * vy;
        if (dt) ot[i] = gi * vt;
        if (s1) of[i] = gi * vf;
    }
}

}  // namespace
}  // namespace capvndf

extern "C" int32_t albedo_view_from_angles(int64_t n, const float* theta_o, const float* phi_o,
                                           float* wox, float* woy, float* woz, void* stream) {
    if (n < 0) return fail(CAPVNDF_ERR_BAD_SIZE, "albedo_view_from_angles: n < 0");
    if (n == 0) return CAPVNDF_OK;
    const void* req[] = {theta_o, phi_o, wox, woy, woz};
    const char* names[] = {"theta_o", "phi_o", "wox", "woy", "woz"};
    for (int i = 0; i < 5; ++i)
        if (int32_t rc = check_array(req[i], names[i])) return rc;
    hipLaunchKernelGGL(k_view_from_angles, dim3(elt_grid(n)), dim3(kEltBlock), 0,
                       as_stream(stream), n, theta_o, phi_o, wox, woy, woz);
    return check_launch("albedo_view_from_angles launch");
}

extern "C" int32_t albedo_apply_jacobian(int64_t n, const float* grad_albedo, const float* d_ax,
                                         const float* d_ay, const float* d_theta_o,
                                         const float* s_f1, const float* s_f5, float* grad_ax,
                                         float* grad_ay, float* grad_theta_o, float* grad_f0,
                                         void* stream) {
    if (n < 0) return fail(CAPVNDF_ERR_BAD_SIZE, "albedo_apply_jacobian: n < 0");
    // every output goes with its input(s): both given or both NULL
    const void* in[] = {d_ax, d_ay, d_theta_o, s_f1, s_f5};
    const void* out[] = {grad_ax, grad_ay, grad_theta_o, grad_f0, grad_f0};
    const char* names[] = {"d_ax", "d_ay", "d_theta_o", "s_f1", "s_f5"};
    for (int i = 0; i < 5; ++i)
        if ((in[i] == nullptr) != (out[i] == nullptr))
            return fail(CAPVNDF_ERR_NULL_PTR,
                        "albedo_apply_jacobian: %s and its gradient output must be given together",
                        names[i]);
    if (n == 0) return CAPVNDF_OK;
    if (int32_t rc = check_array(grad_albedo, "grad_albedo")) return rc;
    const char* onames[] = {"grad_ax", "grad_ay", "grad_theta_o", "grad_f0", "grad_f0"};
    for (int i = 0; i < 5; ++i)
        if (in[i] != nullptr) {
            if (int32_t rc = check_array(in[i], names[i])) return rc;
            if (int32_t rc = check_array(out[i], onames[i])) return rc;
        }
    hipLaunchKernelGGL(k_apply_jacobian, dim3(elt_grid(n)), dim3(kEltBlock), 0, as_stream(stream),
                       n, grad_albedo, d_ax, d_ay, d_theta_o, s_f1, s_f5, grad_ax, grad_ay,
                       grad_theta_o, grad_f0);
    return check_launch("albedo_apply_jacobian launch");
}

// ===========================================================================
// Batch plans.
// ===========================================================================
struct capvndf_batch_plan {
    int device = 0;
    int64_t njobs = 0, nchunks = 0, total_samples = 0;
    capvndf_tiling tiling{};
    int grid = 0;
    int with_grad = 0;
    uint64_t seed = 0;
    const float *wox = nullptr, *woy = nullptr, *woz = nullptr, *ax = nullptr, *ay = nullptr,
                *f0 = nullptr;
    float *albedo = nullptr, *gax = nullptr, *gay = nullptr, *gth = nullptr;
    std::vector<int64_t> nsamp_host;
    // plan-owned device memory: one allocation carved into the tables
    void* dmem = nullptr;
    int32_t* d_chunk_job = nullptr;
    int64_t* d_chunk_pbeg = nullptr;
    int64_t* d_chunk_pend = nullptr;
    int32_t* d_block_chunks = nullptr;
    int32_t* d_job_chunks = nullptr;
    int64_t* d_nsamp = nullptr;
    float* d_partial = nullptr;
    uint64_t* d_rec = nullptr;  // horizon records of the chunks (with_grad)
    float* d_req_ws = nullptr;  // per-request baseline scratch
    uint64_t* d_req_rec = nullptr;
    int32_t* d_counter = nullptr;  // dynamic scheduling
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // recorded after every run; destroy waits for it before freeing
    hipEvent_t done = nullptr;
};

namespace capvndf {
namespace {

bool valid_tiling(const capvndf_tiling& t) {
    return (t.block == 256 || t.block == 512) && t.pairs_per_thread >= kGroup &&
           t.pairs_per_thread <= 4096 && t.pairs_per_thread % kGroup == 0 &&
           t.blocks_per_cu >= 1 && t.blocks_per_cu <= 32 && (t.per_wave == 0 || t.per_wave == 1) &&
           (t.dynamic == 0 || t.dynamic == 1);
}

capvndf_tiling default_tiling() { return capvndf_tiling{256, 32, 8, 0, 0}; }

std::string problem_signature(int device, int64_t njobs, int64_t total, int with_grad) {
    hipDeviceProp_t prop;
    char arch[64] = "unknown";
    int cus = 0;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        snprintf(arch, sizeof(arch), "%s", prop.gcnArchName);
        for (char* p = arch; *p; ++p)
            if (*p == ' ' || *p == ':') *p = '_';
        cus = prop.multiProcessorCount;
    }
    char buf[256];
    snprintf(buf, sizeof(buf), "%s/cu%d/jobs%lld/samples%lld/grad%d", arch, cus, (long long)njobs,
             (long long)total, with_grad);
    return buf;
}

// Tuning cache: text lines
// "<signature> <block> <pairs_per_thread> <blocks_per_cu> <per_wave> <dynamic> <ms>".
bool cache_lookup(const std::string& sig, capvndf_tiling* out) {
    const char* path = getenv("CAPVNDF_TUNE_CACHE");
    if (!path || !*path) return false;
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[512], key[256];
    int b, p, c, w, dy;
    float ms;
    bool found = false;
    // line by line, exactly seven whitespace-separated fields: lines of
    // another layout (an older one without the dynamic field, a truncated
    // write) are skipped
    while (fgets(line, sizeof(line), f)) {
        int fields = 0;
        for (const char* q = line; *q;) {
            while (*q == ' ' || *q == '\t' || *q == '\n' || *q == '\r') ++q;
            if (!*q) break;
            ++fields;
            while (*q && *q != ' ' && *q != '\t' && *q != '\n' && *q != '\r') ++q;
        }
        if (fields != 7 ||
            sscanf(line, "%255s %d %d %d %d %d %f", key, &b, &p, &c, &w, &dy, &ms) != 7)
            continue;
        capvndf_tiling t{b, p, c, w, dy};
        if (sig == key && valid_tiling(t)) {
            *out = t;  // last matching line wins
            found = true;
        }
    }
    fclose(f);
    return found;
}

void cache_store(const std::string& sig, const capvndf_tiling& t, float ms) {
    const char* path = getenv("CAPVNDF_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d %d %d %d %d %.6f\n", sig.c_str(), t.block, t.pairs_per_thread,
            t.blocks_per_cu, t.per_wave, t.dynamic, ms);
    fclose(f);
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Threads of a chunk's owner: a wavefront per wave, else the block.
int32_t owner_threads(const capvndf_tiling& t) { return t.per_wave ? 64 : t.block; }

int32_t enqueue_batch(capvndf_batch_plan* p, hipStream_t st) {
    const int g = p->with_grad;
    const uint32_t k0 = key_lo(p->seed), k1 = key_hi(p->seed);
    const dim3 grid((unsigned)p->grid), block((unsigned)p->tiling.block);
    const bool dyn = p->tiling.dynamic != 0;
    if (dyn) {
        hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, p->d_counter);
        if (int32_t rc = check_launch("batch counter reset")) return rc;
    }
#define CAPVNDF_LAUNCH_BATCH(K, B, G, D)                                                            \
    hipLaunchKernelGGL((K<B, G, D>), grid, block, 0, st, p->wox, p->woy, p->woz, p->ax, p->ay,    \
                       p->f0, p->d_nsamp, p->d_chunk_job, p->d_chunk_pbeg, p->d_chunk_pend,        \
                       p->d_block_chunks, p->d_counter, (int32_t)p->nchunks, k0, k1, p->d_partial, \
                       p->d_rec)
#define CAPVNDF_LAUNCH_BATCH_D(K, B, G)                                                             \
    do {                                                                                            \
        if (dyn) CAPVNDF_LAUNCH_BATCH(K, B, G, true);                                               \
        else CAPVNDF_LAUNCH_BATCH(K, B, G, false);                                                  \
    } while (0)
    if (p->tiling.per_wave) {
        if (p->tiling.block == 256) {
            if (g) CAPVNDF_LAUNCH_BATCH_D(k_batch_wave, 256, true);
            else CAPVNDF_LAUNCH_BATCH_D(k_batch_wave, 256, false);
        } else {
            if (g) CAPVNDF_LAUNCH_BATCH_D(k_batch_wave, 512, true);
            else CAPVNDF_LAUNCH_BATCH_D(k_batch_wave, 512, false);
        }
    } else if (p->tiling.block == 256) {
        if (g) CAPVNDF_LAUNCH_BATCH_D(k_batch, 256, true);
        else CAPVNDF_LAUNCH_BATCH_D(k_batch, 256, false);
    } else {
        if (g) CAPVNDF_LAUNCH_BATCH_D(k_batch, 512, true);
        else CAPVNDF_LAUNCH_BATCH_D(k_batch, 512, false);
    }
#undef CAPVNDF_LAUNCH_BATCH_D
#undef CAPVNDF_LAUNCH_BATCH
    if (int32_t rc = check_launch("batch kernel launch")) return rc;
    if (g && p->nchunks > 0) {  // a plan of empty jobs has no chunks, and nothing to fix
        launch_fix_batch(p->nchunks, owner_threads(p->tiling), p->wox, p->woy, p->woz, p->ax,
                         p->ay, p->f0, p->d_nsamp, p->d_chunk_job, p->d_chunk_pbeg,
                         p->d_chunk_pend, k0, k1, p->d_rec, p->d_partial, st);
        if (int32_t rc = check_launch("batch fix launch")) return rc;
    }
    if (g)
        hipLaunchKernelGGL(k_finish<4>, dim3(finish_grid(p->njobs)), dim3(kFinishBlock), 0, st,
                           p->njobs, p->d_partial, 0, p->d_job_chunks, p->d_nsamp, nullptr,
                           p->albedo, p->gax, p->gay, p->gth);
    else
        hipLaunchKernelGGL(k_finish<1>, dim3(finish_grid(p->njobs)), dim3(kFinishBlock), 0, st,
                           p->njobs, p->d_partial, 0, p->d_job_chunks, p->d_nsamp, nullptr,
                           p->albedo, nullptr, nullptr, nullptr);
    return check_launch("batch finish launch");
}

void destroy_plan(capvndf_batch_plan* p) {
    if (!p) return;
    // a run still in flight reads and writes the memory freed below
    if (p->done) {
        (void)hipEventSynchronize(p->done);
        (void)hipEventDestroy(p->done);
    }
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->dmem) (void)hipFree(p->dmem);
    delete p;
}

int32_t create_plan(int64_t njobs, const float* wox, const float* woy, const float* woz,
                    const float* ax, const float* ay, const float* f0, const int64_t* nsamples_host,
                    uint64_t seed, int32_t with_grad, float* albedo, float* grad_ax,
                    float* grad_ay, float* grad_theta_o, const capvndf_tiling* tiling,
                    capvndf_batch_plan** out) {
    if (out == nullptr) return fail(CAPVNDF_ERR_NULL_PTR, "albedo_batch_plan_create: out is NULL");
    *out = nullptr;
    if (njobs < 1 || njobs > ((int64_t)1 << 31) - 2)
        return fail(CAPVNDF_ERR_BAD_SIZE, "albedo_batch_plan_create: njobs must be in [1, 2^31 - 2]");
    if (nsamples_host == nullptr)
        return fail(CAPVNDF_ERR_NULL_PTR, "albedo_batch_plan_create: nsamples_host is NULL");
    {
        const void* req[] = {wox, woy, woz, ax, ay};
        const char* names[] = {"wox", "woy", "woz", "ax", "ay"};
        for (int i = 0; i < 5; ++i)
            if (int32_t rc = check_array(req[i], names[i])) return rc;
    }
    if (int32_t rc = check_array(albedo, "albedo")) return rc;
    if (f0 != nullptr)
        if (int32_t rc = check_array(f0, "f0")) return rc;
    if (with_grad != 0 && with_grad != 1)
        return fail(CAPVNDF_ERR_BAD_ARG, "albedo_batch_plan_create: with_grad must be 0 or 1");
    if (with_grad) {
        if (int32_t rc = check_array(grad_ax, "grad_ax")) return rc;
        if (int32_t rc = check_array(grad_ay, "grad_ay")) return rc;
        if (int32_t rc = check_array(grad_theta_o, "grad_theta_o")) return rc;
    }
    int64_t total = 0, max_n = 0;
    for (int64_t j = 0; j < njobs; ++j) {
        const int64_t n = nsamples_host[j];
        if (n < 0 || n >= ((int64_t)1 << 40))
            return fail(CAPVNDF_ERR_BAD_SIZE, "albedo_batch_plan_create: nsamples[%lld] out of [0, 2^40)",
                        (long long)j);
        total += n;
        max_n = std::max(max_n, n);
    }
    capvndf_tiling t = default_tiling();
    int device = 0;
    if (int32_t rc = check_hip(hipGetDevice(&device), "hipGetDevice")) return rc;
    if (tiling) {
        if (!valid_tiling(*tiling))
            return fail(CAPVNDF_ERR_BAD_ARG,
                        "albedo_batch_plan_create: invalid tiling (block 256|512, pairs_per_thread "
                        "a multiple of 8 in [8, 4096], blocks_per_cu in [1, 32], per_wave 0|1, "
                        "dynamic 0|1)");
        t = *tiling;
    } else {
        (void)cache_lookup(problem_signature(device, njobs, total, with_grad), &t);
    }
    int cus = 0;
    if (int32_t rc = check_hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device),
                               "hipDeviceGetAttribute"))
        return rc;

    // Chunk table: job-major, pair ranges of chunk_pairs (one block's or, per
    // wave, one wavefront's lanes times pairs_per_thread).
    const int64_t chunk_pairs = (int64_t)(t.per_wave ? 64 : t.block) * t.pairs_per_thread;
    // count first: chunk indices are int32 on the device, and the tables are
    // sized exactly (no growth while they are built)
    int64_t count = 0;
    for (int64_t j = 0; j < njobs; ++j)
        count += ((nsamples_host[j] + 1) / 2 + chunk_pairs - 1) / chunk_pairs;
    if (count > (int64_t)0x7ffffffe)
        return fail(CAPVNDF_ERR_BAD_SIZE,
                    "albedo_batch_plan_create: %lld chunks of %lld sample pairs exceed 2^31 - 2; "
                    "raise pairs_per_thread or split the jobs over several plans",
                    (long long)count, (long long)chunk_pairs);
    std::vector<int32_t> chunk_job;
    std::vector<int64_t> pbeg, pend;
    chunk_job.reserve((size_t)count);
    pbeg.reserve((size_t)count);
    pend.reserve((size_t)count);
    std::vector<int32_t> job_chunks((size_t)njobs + 1, 0);
    for (int64_t j = 0; j < njobs; ++j) {
        job_chunks[j] = (int32_t)chunk_job.size();
        const int64_t np = (nsamples_host[j] + 1) / 2;
        for (int64_t b = 0; b < np; b += chunk_pairs) {
            chunk_job.push_back((int32_t)j);
            pbeg.push_back(b);
            pend.push_back(std::min(b + chunk_pairs, np));
        }
    }
    job_chunks[njobs] = (int32_t)chunk_job.size();
    const int64_t nchunks = (int64_t)chunk_job.size();

    // Static partition of the chunks over the persistent grid's owners (its
    // blocks, or its wavefronts per wave), balanced by pairs.
    const int64_t waves_per_block = t.per_wave ? t.block / 64 : 1;
    int64_t grid = std::max<int64_t>(1, (int64_t)cus * t.blocks_per_cu);
    if (nchunks > 0) grid = std::min<int64_t>(grid, (nchunks + waves_per_block - 1) / waves_per_block);
    const int64_t owners = grid * waves_per_block;
    std::vector<int32_t> block_chunks((size_t)owners + 1, 0);
    {
        double sum = 0.0;
        for (int64_t c = 0; c < nchunks; ++c) sum += (double)(pend[c] - pbeg[c]);
        double acc = 0.0;
        int64_t c = 0;
        for (int64_t b = 0; b < owners; ++b) {
            block_chunks[b] = (int32_t)c;
            const double target = sum * (double)(b + 1) / (double)owners;
            while (c < nchunks && (acc + 0.5 * (double)(pend[c] - pbeg[c]) <= target || b == owners - 1)) {
                acc += (double)(pend[c] - pbeg[c]);
                ++c;
            }
        }
        block_chunks[owners] = (int32_t)nchunks;
    }

    // Device memory: tables, partials, per-request scratch.
    const int nacc = with_grad ? 4 : 1;
    const int64_t max_cpc = std::max<int64_t>(1, cell_chunks(max_n));
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    const size_t o_cj = carve(sizeof(int32_t) * std::max<int64_t>(nchunks, 1));
    const size_t o_pb = carve(sizeof(int64_t) * std::max<int64_t>(nchunks, 1));
    const size_t o_pe = carve(sizeof(int64_t) * std::max<int64_t>(nchunks, 1));
    const size_t o_bc = carve(sizeof(int32_t) * (size_t)(owners + 1));
    const size_t o_jc = carve(sizeof(int32_t) * (size_t)(njobs + 1));
    const size_t o_ns = carve(sizeof(int64_t) * (size_t)njobs);
    const size_t o_pa = carve(sizeof(float) * 2 * nacc * (size_t)std::max<int64_t>(nchunks, 1));
    const int rec_words = owner_threads(t) / 64;
    const size_t o_rc = carve(with_grad ? rec_bytes(std::max<int64_t>(nchunks, 1), rec_words) : 8);
    const size_t o_rw = carve(sizeof(float) * 8 * (size_t)max_cpc);
    const size_t o_rr = carve(with_grad ? rec_bytes(max_cpc, kLutBlock / 64) : 8);
    const size_t o_ct = carve(sizeof(int32_t));
    capvndf_batch_plan* p = new capvndf_batch_plan();
    if (int32_t rc = check_hip(hipMalloc(&p->dmem, off), "hipMalloc (batch plan)")) {
        p->dmem = nullptr;
        destroy_plan(p);
        return rc;
    }
    char* base = static_cast<char*>(p->dmem);
    p->d_chunk_job = reinterpret_cast<int32_t*>(base + o_cj);
    p->d_chunk_pbeg = reinterpret_cast<int64_t*>(base + o_pb);
    p->d_chunk_pend = reinterpret_cast<int64_t*>(base + o_pe);
    p->d_block_chunks = reinterpret_cast<int32_t*>(base + o_bc);
    p->d_job_chunks = reinterpret_cast<int32_t*>(base + o_jc);
    p->d_nsamp = reinterpret_cast<int64_t*>(base + o_ns);
    p->d_partial = reinterpret_cast<float*>(base + o_pa);
    p->d_rec = reinterpret_cast<uint64_t*>(base + o_rc);
    p->d_req_ws = reinterpret_cast<float*>(base + o_rw);
    p->d_req_rec = reinterpret_cast<uint64_t*>(base + o_rr);
    p->d_counter = reinterpret_cast<int32_t*>(base + o_ct);
    int32_t rc = CAPVNDF_OK;
    if (nchunks > 0) {
        if (!rc) rc = check_hip(hipMemcpy(p->d_chunk_job, chunk_job.data(), sizeof(int32_t) * nchunks, hipMemcpyHostToDevice), "hipMemcpy");
        if (!rc) rc = check_hip(hipMemcpy(p->d_chunk_pbeg, pbeg.data(), sizeof(int64_t) * nchunks, hipMemcpyHostToDevice), "hipMemcpy");
        if (!rc) rc = check_hip(hipMemcpy(p->d_chunk_pend, pend.data(), sizeof(int64_t) * nchunks, hipMemcpyHostToDevice), "hipMemcpy");
    }
    if (!rc) rc = check_hip(hipMemcpy(p->d_block_chunks, block_chunks.data(), sizeof(int32_t) * (owners + 1), hipMemcpyHostToDevice), "hipMemcpy");
    if (!rc) rc = check_hip(hipMemcpy(p->d_job_chunks, job_chunks.data(), sizeof(int32_t) * (njobs + 1), hipMemcpyHostToDevice), "hipMemcpy");
    if (!rc) rc = check_hip(hipMemcpy(p->d_nsamp, nsamples_host, sizeof(int64_t) * njobs, hipMemcpyHostToDevice), "hipMemcpy");
    if (rc) {
        destroy_plan(p);
        return rc;
    }
    p->device = device;
    p->njobs = njobs;
    p->nchunks = nchunks;
    p->total_samples = total;
    p->tiling = t;
    p->grid = (int)grid;
    p->with_grad = with_grad;
    p->seed = seed;
    p->wox = wox; p->woy = woy; p->woz = woz; p->ax = ax; p->ay = ay; p->f0 = f0;
    p->albedo = albedo;
    p->gax = with_grad ? grad_ax : nullptr;
    p->gay = with_grad ? grad_ay : nullptr;
    p->gth = with_grad ? grad_theta_o : nullptr;
    p->nsamp_host.assign(nsamples_host, nsamples_host + njobs);

    // Capture the launch sequence once on a private stream.
    hipStream_t cap = nullptr;
    rc = check_hip(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "hipStreamCreateWithFlags");
    if (!rc) rc = check_hip(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    if (!rc) {
        const int32_t rl = enqueue_batch(p, cap);
        hipGraph_t g = nullptr;
        const int32_t re = check_hip(hipStreamEndCapture(cap, &g), "hipStreamEndCapture");
        p->graph = g;
        rc = rl ? rl : re;
    }
    if (!rc) rc = check_hip(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    if (!rc) rc = check_hip(hipEventCreateWithFlags(&p->done, hipEventDisableTiming), "hipEventCreateWithFlags");
    if (cap) (void)hipStreamDestroy(cap);
    if (rc) {
        destroy_plan(p);
        return rc;
    }
    *out = p;
    return CAPVNDF_OK;
}

}  // namespace
}  // namespace capvndf

extern "C" int32_t albedo_batch_plan_create(int64_t njobs, const float* wox, const float* woy,
                                            const float* woz, const float* ax, const float* ay,
                                            const float* f0, const int64_t* nsamples_host,
                                            uint64_t seed, int32_t with_grad, float* albedo,
                                            float* grad_ax, float* grad_ay, float* grad_theta_o,
                                            const capvndf_tiling* tiling, void* stream,
                                            capvndf_batch_plan** out) {
    (void)stream;  // capture happens on a private stream; replays use the caller's
    return create_plan(njobs, wox, woy, woz, ax, ay, f0, nsamples_host, seed, with_grad, albedo,
                       grad_ax, grad_ay, grad_theta_o, tiling, out);
}

namespace {
// A plan's pointers and graph belong to the device it was created on.
int32_t check_plan_device(const capvndf_batch_plan* p, const char* who) {
    int dev = 0;
    if (int32_t rc = check_hip(hipGetDevice(&dev), "hipGetDevice")) return rc;
    if (dev != p->device)
        return fail(CAPVNDF_ERR_BAD_ARG, "%s: the plan belongs to device %d, current device is %d",
                    who, p->device, dev);
    return CAPVNDF_OK;
}
}  // namespace

extern "C" int32_t albedo_batch_run(capvndf_batch_plan* plan, void* stream) {
    if (plan == nullptr) return fail(CAPVNDF_ERR_NULL_PTR, "albedo_batch_run: plan is NULL");
    if (int32_t rc = check_plan_device(plan, "albedo_batch_run")) return rc;
    if (int32_t rc = check_hip(hipGraphLaunch(plan->exec, as_stream(stream)), "hipGraphLaunch"))
        return rc;
    return check_hip(hipEventRecord(plan->done, as_stream(stream)), "hipEventRecord");
}

extern "C" int32_t albedo_batch_run_per_request(capvndf_batch_plan* p, void* stream) {
    if (p == nullptr) return fail(CAPVNDF_ERR_NULL_PTR, "albedo_batch_run_per_request: plan is NULL");
    if (int32_t rc = check_plan_device(p, "albedo_batch_run_per_request")) return rc;
    // one kLutBlock block per chunk of a job: each launch must fit a 32-bit
    // work-item count; checked for every job before anything is enqueued
    for (int64_t j = 0; j < p->njobs; ++j)
        if (cell_chunks(p->nsamp_host[j]) > kMaxBlocks)
            return fail(CAPVNDF_ERR_BAD_SIZE,
                        "albedo_batch_run_per_request: job %lld has %lld samples, more than one "
                        "launch of this path covers (2^24 - 1 chunks of %llu samples)",
                        (long long)j, (long long)p->nsamp_host[j],
                        (unsigned long long)(2 * kLutChunkPairs));
    const hipStream_t st = as_stream(stream);
    const uint32_t k0 = key_lo(p->seed), k1 = key_hi(p->seed);
    for (int64_t j = 0; j < p->njobs; ++j) {
        // the table kernels on one cell, one slot per chunk of the job
        const int32_t cpc = (int32_t)cell_chunks(p->nsamp_host[j]);
        const int32_t slots = std::max<int32_t>(cpc, 1);
        const float* f0 = p->f0 ? p->f0 + j : nullptr;
        const int64_t* nj = p->d_nsamp + j;
        if (p->with_grad) {
            if (cpc > 0) {
                hipLaunchKernelGGL(k_albedo_adj<true>, dim3((unsigned)cpc), dim3(kLutBlock), 0, st,
                                   p->wox + j, p->woy + j, p->woz + j, p->ax + j, p->ay + j, f0,
                                   nj, slots, (uint32_t)j, k0, k1, p->d_req_ws, p->d_req_rec);
                launch_table_fix<true>(1, slots, p->wox + j, p->woy + j, p->woz + j, p->ax + j,
                                       p->ay + j, f0, nj, (uint32_t)j, k0, k1, p->d_req_rec,
                                       p->d_req_ws, st);
            }
            hipLaunchKernelGGL(k_finish<4>, dim3(1), dim3(kFinishBlock), 0, st, (int64_t)1,
                               p->d_req_ws, slots, nullptr, nj, nullptr, p->albedo + j,
                               p->gax + j, p->gay + j, p->gth + j);
        } else {
            if (cpc > 0)
                hipLaunchKernelGGL(k_albedo_fwd<1>, dim3((unsigned)cpc), dim3(kLutBlock), 0, st,
                                   p->wox + j, p->woy + j, p->woz + j, p->ax + j, p->ay + j, f0,
                                   nj, slots, (uint32_t)j, k0, k1, p->d_req_ws);
            hipLaunchKernelGGL(k_finish<1>, dim3(1), dim3(kFinishBlock), 0, st, (int64_t)1,
                               p->d_req_ws, slots, nullptr, nj, nullptr, p->albedo + j, nullptr,
                               nullptr, nullptr);
        }
    }
    if (int32_t rc = check_launch("albedo_batch_run_per_request launch")) return rc;
    return check_hip(hipEventRecord(p->done, st), "hipEventRecord");
}

extern "C" int32_t albedo_batch_plan_info(const capvndf_batch_plan* plan, capvndf_tiling* tiling,
                                          int64_t* nchunks, int64_t* total_samples) {
    if (plan == nullptr) return fail(CAPVNDF_ERR_NULL_PTR, "albedo_batch_plan_info: plan is NULL");
    if (tiling) *tiling = plan->tiling;
    if (nchunks) *nchunks = plan->nchunks;
    if (total_samples) *total_samples = plan->total_samples;
    return CAPVNDF_OK;
}

extern "C" void albedo_batch_plan_destroy(capvndf_batch_plan* plan) { destroy_plan(plan); }

extern "C" int32_t albedo_batch_autotune(int64_t njobs, const float* wox, const float* woy,
                                         const float* woz, const float* ax, const float* ay,
                                         const float* f0, const int64_t* nsamples_host,
                                         uint64_t seed, int32_t with_grad, float* albedo,
                                         float* grad_ax, float* grad_ay, float* grad_theta_o,
                                         void* stream, capvndf_tiling* best, float* best_ms) {
    if (best == nullptr) return fail(CAPVNDF_ERR_NULL_PTR, "albedo_batch_autotune: best is NULL");
    const hipStream_t st = as_stream(stream);
    const int blocks[] = {256, 512};
    const int ppts[] = {8, 16, 32, 64, 128};
    const int bpcs[] = {2, 4, 8, 16};
    const int modes[] = {0, 1};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int32_t rc = check_hip(hipEventCreate(&e0), "hipEventCreate");
    if (!rc) rc = check_hip(hipEventCreate(&e1), "hipEventCreate");
    float best_t = 3.4e38f;
    capvndf_tiling best_tiling = default_tiling();
    int tried = 0;
    int32_t size_rc = CAPVNDF_OK;  // kept for when no candidate can be built
    int64_t total = 0;
    for (int64_t j = 0; j < njobs && nsamples_host; ++j) total += nsamples_host[j];
    for (int dyn = 0; dyn < 2; ++dyn)
    for (int mode : modes)
    for (int b : blocks)
    for (int ppt : ppts)
    for (int bpc : bpcs) {
        if (rc) break;
        if (b == 512 && bpc > 8) continue;
        if (mode == 0 && ppt > 64) continue;
        capvndf_tiling t{b, ppt, bpc, mode, dyn};
        capvndf_batch_plan* p = nullptr;
        rc = create_plan(njobs, wox, woy, woz, ax, ay, f0, nsamples_host, seed, with_grad, albedo,
                         grad_ax, grad_ay, grad_theta_o, &t, &p);
        if (rc == CAPVNDF_ERR_BAD_SIZE) {  // e.g. too many chunks at this size: skip it
            size_rc = rc;
            rc = CAPVNDF_OK;
            continue;
        }
        if (rc) break;
        ++tried;
        rc = check_hip(hipGraphLaunch(p->exec, st), "hipGraphLaunch");  // warm-up
        const int reps = 3;
        if (!rc) rc = check_hip(hipEventRecord(e0, st), "hipEventRecord");
        for (int r = 0; r < reps && !rc; ++r)
            rc = check_hip(hipGraphLaunch(p->exec, st), "hipGraphLaunch");
        if (!rc) rc = check_hip(hipEventRecord(e1, st), "hipEventRecord");
        if (!rc) rc = check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0.0f;
        if (!rc) rc = check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        if (rc) (void)hipStreamSynchronize(st);  // no replay may be pending when it is freed
        destroy_plan(p);
        if (!rc && ms / reps < best_t) {
            best_t = ms / reps;
            best_tiling = t;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (tried == 0) return size_rc;  // its message is the last failure's
    *best = best_tiling;
    if (best_ms) *best_ms = best_t;
    int device = 0;
    if (hipGetDevice(&device) == hipSuccess)
        cache_store(problem_signature(device, njobs, total, with_grad), best_tiling, best_t);
    return CAPVNDF_OK;
}
