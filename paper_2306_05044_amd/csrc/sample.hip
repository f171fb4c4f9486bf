// Streaming VNDF sampling and pdf kernels, random-number hooks, the
// register-resident microbenchmark and the streaming-bandwidth probe.
//
// Layout: structure of arrays in HBM.  The vector path gives each lane groups
// of four consecutive tuples, so every array is read and written with 16-byte
// accesses per lane (fully coalesced dwordx4, non-temporal: nothing is
// reused), and each group of four tuples takes exactly two Philox blocks.
#include "common.hpp"
#include "device_math.hpp"
#include "stream_io.hpp"

namespace capvndf {
namespace {

// Launch shapes of the evaluation kernels, whose outputs are small next to
// their inputs (pdf: 32 B in, 4 B out; inverse map: 32 B in, 8 B out): vec4
// groups per lane, threads per block (wavefront tiles) and whether the
// outputs go through the cache.  Measured at 2^26: a cached pdf store is 4 %
// faster than a non-temporal one, while the inverse map's two outputs are
// 6 % faster non-temporal; 256-thread blocks beat 128 by 3 % (pdf) and 4 %
// (inverse); lane-interleaved groups were no better.
#ifndef CAPVNDF_PDF_GROUPS
#define CAPVNDF_PDF_GROUPS 4
#endif
#ifndef CAPVNDF_PDF_CACHED
#define CAPVNDF_PDF_CACHED 1
#endif
#ifndef CAPVNDF_INVERSE_GROUPS
#define CAPVNDF_INVERSE_GROUPS 4
#endif
#ifndef CAPVNDF_INVERSE_CACHED
#define CAPVNDF_INVERSE_CACHED 0
#endif
// vec4 groups per lane of the double-precision sampler, whose registers per
// tuple are about twice the FP32 sampler's.  Measured at 2^26: one group
// 0.413 ms, two 0.450 ms, four 0.427 ms (the FP32 sampler: 0.404-0.407 ms).
#ifndef CAPVNDF_F64_GROUPS
#define CAPVNDF_F64_GROUPS 1
#endif
constexpr int kF64Groups = CAPVNDF_F64_GROUPS;
#ifndef CAPVNDF_PDF_BLOCK
#define CAPVNDF_PDF_BLOCK 256
#endif
#ifndef CAPVNDF_INVERSE_BLOCK
#define CAPVNDF_INVERSE_BLOCK 256
#endif
constexpr int kPdfBlock = CAPVNDF_PDF_BLOCK;
constexpr int kInverseBlock = CAPVNDF_INVERSE_BLOCK;
constexpr int kPdfGroups = CAPVNDF_PDF_GROUPS;
constexpr bool kPdfCached = CAPVNDF_PDF_CACHED != 0;
constexpr int kInverseGroups = CAPVNDF_INVERSE_GROUPS;
constexpr bool kInverseCached = CAPVNDF_INVERSE_CACHED != 0;

// One tuple: general sampler with the chosen hemisphere routine.  Inputs
// outside the domain are replaced by harmless ones and the outputs selected
// afterwards, so the vector path stays branch-free.
template <int METHOD, bool WITH_PDF>
__device__ __forceinline__ void sample_one(float wx, float wy, float wz, float ax, float ay,
                                           float u1, float u2, float& hx, float& hy, float& hz,
                                           float& pdf) {
    const bool ok = (wz > 0.0f) && (ax > 0.0f) && (ay > 0.0f);
    if (!ok) {
        wx = 0.0f; wy = 0.0f; wz = 1.0f; ax = 1.0f; ay = 1.0f;
    }
    if (METHOD == CAPVNDF_CAP_F64) {
        float p64 = 0.0f;
        cap_sample_f64<WITH_PDF>(wx, wy, wz, ax, ay, u1, u2, hx, hy, hz, p64);
        if (!ok) {
            hx = 0.0f; hy = 0.0f; hz = 1.0f;
        }
        pdf = ok ? p64 : 0.0f;
        return;
    }
    const Stretched s = stretch(wx, wy, wz, ax, ay);
    float p = 0.0f;
    Normal n;
    if (METHOD == CAPVNDF_CAP) {
        const CapSample c = cap_sample(s, u1, u2);
        n = unstretch(c.hsx, c.hsy, c.hsz, ax, ay);
        if (WITH_PDF) p = cap_pdf(s, c, n, ax, ay);
    } else {
        const DiskSample d = disk2018_sample(s, u1, u2);
        n = unstretch(d.mx, d.my, d.mz, ax, ay);
        if (WITH_PDF) p = disk_pdf(s, d, n, ax, ay);
    }
    hx = ok ? n.hx : 0.0f;
    hy = ok ? n.hy : 0.0f;
    hz = ok ? n.hz : 1.0f;
    pdf = ok ? p : 0.0f;
}

__device__ __forceinline__ void stream_u(uint64_t k, uint32_t key0, uint32_t key1, float& u1,
                                         float& u2) {
    const Words w = philox_pair(k >> 1, 0u, kTagSample, key0, key1);
    const bool odd = (k & 1u) != 0;
    u1 = unit24(odd ? w.w2 : w.w0);
    u2 = unit24(odd ? w.w3 : w.w1);
}

// Vector path (index_base even, arrays 16-byte aligned).  A block owns a tile
// of kBlock * 4 * G consecutive tuples and each lane G groups of
// four (see group_start: every wavefront reads a contiguous run per array).
// All loads of a lane are issued before any arithmetic to keep enough bytes
// in flight.  Groups that straddle n finish their tuples one by one.
template <int METHOD, bool EXPLICIT_U, bool WITH_PDF, int G = kGroups>
__global__ __launch_bounds__(kBlock) void k_sample_v4(
    int64_t n, const float* __restrict__ wix, const float* __restrict__ wiy,
    const float* __restrict__ wiz, const float* __restrict__ ax, const float* __restrict__ ay,
    const float* __restrict__ u1p, const float* __restrict__ u2p, uint64_t index_base,
    uint32_t key0, uint32_t key1, float* __restrict__ hx, float* __restrict__ hy,
    float* __restrict__ hz, float* __restrict__ pdf) {
    const int64_t tile = (int64_t)blockIdx.x * kBlock * 4 * G;
    f4 x[G], y[G], z[G], a[G], b[G], r1[G], r2[G];
    load_groups(x, wix, tile, n);
    load_groups(y, wiy, tile, n);
    load_groups(z, wiz, tile, n);
    load_groups(a, ax, tile, n);
    load_groups(b, ay, tile, n);
    if (EXPLICIT_U) {
        load_groups(r1, u1p, tile, n);
        load_groups(r2, u2p, tile, n);
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t i0 = group_start<G>(tile, g);
        if (i0 + 4 <= n) {
            if (!EXPLICIT_U) {
                const uint64_t pair = (index_base >> 1) + (uint64_t)(i0 >> 1);
                const Words w0 = philox_pair(pair, 0u, kTagSample, key0, key1);
                const Words w1 = philox_pair(pair + 1, 0u, kTagSample, key0, key1);
                r1[g] = f4{unit24(w0.w0), unit24(w0.w2), unit24(w1.w0), unit24(w1.w2)};
                r2[g] = f4{unit24(w0.w1), unit24(w0.w3), unit24(w1.w1), unit24(w1.w3)};
            }
            f4 ox, oy, oz, op;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float hxj, hyj, hzj, pj;
                sample_one<METHOD, WITH_PDF>(x[g][j], y[g][j], z[g][j], a[g][j], b[g][j],
                                             r1[g][j], r2[g][j], hxj, hyj, hzj, pj);
                ox[j] = hxj; oy[j] = hyj; oz[j] = hzj; op[j] = pj;
            }
            store4(hx + i0, ox);
            store4(hy + i0, oy);
            store4(hz + i0, oz);
            if (WITH_PDF) store4(pdf + i0, op);
        } else {
            for (int64_t i = i0; i < n && i < i0 + 4; ++i) {
                float q1, q2;
                if (EXPLICIT_U) {
                    q1 = u1p[i]; q2 = u2p[i];
                } else {
                    stream_u(index_base + (uint64_t)i, key0, key1, q1, q2);
                }
                float hxi, hyi, hzi, pi;
                sample_one<METHOD, WITH_PDF>(wix[i], wiy[i], wiz[i], ax[i], ay[i], q1, q2, hxi,
                                             hyi, hzi, pi);
                hx[i] = hxi; hy[i] = hyi; hz[i] = hzi;
                if (WITH_PDF) pdf[i] = pi;
            }
        }
    }
}

// Scalar path (any 4-byte alignment, any index_base): one tuple per lane.
template <int METHOD, bool EXPLICIT_U, bool WITH_PDF>
__global__ __launch_bounds__(kBlock) void k_sample_scalar(
    int64_t n, const float* __restrict__ wix, const float* __restrict__ wiy,
    const float* __restrict__ wiz, const float* __restrict__ ax, const float* __restrict__ ay,
    const float* __restrict__ u1p, const float* __restrict__ u2p, uint64_t index_base,
    uint32_t key0, uint32_t key1, float* __restrict__ hx, float* __restrict__ hy,
    float* __restrict__ hz, float* __restrict__ pdf) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    float r1, r2;
    if (EXPLICIT_U) {
        r1 = u1p[i]; r2 = u2p[i];
    } else {
        stream_u(index_base + (uint64_t)i, key0, key1, r1, r2);
    }
    float hxi, hyi, hzi, pi;
    sample_one<METHOD, WITH_PDF>(wix[i], wiy[i], wiz[i], ax[i], ay[i], r1, r2, hxi, hyi, hzi,
                                 pi);
    hx[i] = hxi; hy[i] = hyi; hz[i] = hzi;
    if (WITH_PDF) pdf[i] = pi;
}

// pdf of Eq. (1) at a given unit h: G1(wi) = 2 w_z / (l + w_z) with
// l = |M^-1 wi|, D(h) = 1 / (pi ax ay k^2) with k = |M^T h|^2, so
// pdf = 2 (wi.h) / ((l + w_z) pi ax ay k^2).  Evaluated in double: the
// three products of wi.h are exact there (24 x 24 bits) and are summed with
// error-free transformations, so the dot product, which cancels near
// grazing, keeps its full relative accuracy; the other factors are sums of
// squares.  With K = k ax^2 ay^2 = (hx ay)^2 + (hy ax)^2 + (hz ax ay)^2,
// pdf = 2 (wi.h) ax^3 ay^3 / ((l + w_z) pi K^2): one reciprocal.  The kernel
// is bound by HBM traffic, which hides the double arithmetic.
__device__ __forceinline__ double two_sum(double a, double b, double& err) {
    const double s = a + b;
    const double bb = s - a;
    err = (a - (s - bb)) + (b - bb);
    return s;
}

__device__ __forceinline__ float pdf_one(float wxf, float wyf, float wzf, float hxf, float hyf,
                                         float hzf, float axf, float ayf) {
    const bool ok0 = (wzf > 0.0f) && (axf > 0.0f) && (ayf > 0.0f) && (hzf > 0.0f);
    if (!ok0) {
        wzf = 1.0f; axf = 1.0f; ayf = 1.0f; hzf = 1.0f;
    }
    const double wx = wxf, wy = wyf, wz = wzf, hx = hxf, hy = hyf, hz = hzf;
    const double ax = axf, ay = ayf;
    double e1, e2;
    const double s12 = two_sum(wx * hx, wy * hy, e1);
    const double s = two_sum(s12, wz * hz, e2);
    const double d = s + (e1 + e2);
    const double px = ax * wx, py = ay * wy;
    const double l2 = __builtin_fma(px, px, __builtin_fma(py, py, wz * wz));
    const double l = l2 * rsq_f64(l2);
    const double axy = ax * ay;
    const double kx = hx * ay, ky = hy * ax, kz = hz * axy;
    const double K = __builtin_fma(kx, kx, __builtin_fma(ky, ky, kz * kz));
    const double p = 2.0 * d * (axy * axy * axy) * rcp_f64((l + wz) * kPiD * K * K);
    return (ok0 && d > 0.0) ? (float)p : 0.0f;
}

template <int G, bool CACHED_OUT, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_pdf_v4(
    int64_t n, const float* __restrict__ wix, const float* __restrict__ wiy,
    const float* __restrict__ wiz, const float* __restrict__ hxp, const float* __restrict__ hyp,
    const float* __restrict__ hzp, const float* __restrict__ ax, const float* __restrict__ ay,
    float* __restrict__ pdf) {
    const int64_t tile = (int64_t)blockIdx.x * BLOCK * 4 * G;
    f4 x[G], y[G], z[G], hx[G], hy[G], hz[G], a[G], b[G];
    load_groups<G, BLOCK, true>(x, wix, tile, n);
    load_groups<G, BLOCK, true>(y, wiy, tile, n);
    load_groups<G, BLOCK, true>(z, wiz, tile, n);
    load_groups<G, BLOCK, true>(hx, hxp, tile, n);
    load_groups<G, BLOCK, true>(hy, hyp, tile, n);
    load_groups<G, BLOCK, true>(hz, hzp, tile, n);
    load_groups<G, BLOCK, true>(a, ax, tile, n);
    load_groups<G, BLOCK, true>(b, ay, tile, n);
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t i0 = group_start<G, BLOCK, true>(tile, g);
        if (i0 + 4 <= n) {
            f4 o;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                o[j] = pdf_one(x[g][j], y[g][j], z[g][j], hx[g][j], hy[g][j], hz[g][j], a[g][j],
                               b[g][j]);
            if (CACHED_OUT) store4_cached(pdf + i0, o); else store4(pdf + i0, o);
        } else {
            for (int64_t i = i0; i < n && i < i0 + 4; ++i)
                pdf[i] = pdf_one(wix[i], wiy[i], wiz[i], hxp[i], hyp[i], hzp[i], ax[i], ay[i]);
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_pdf_scalar(
    int64_t n, const float* __restrict__ wix, const float* __restrict__ wiy,
    const float* __restrict__ wiz, const float* __restrict__ hxp, const float* __restrict__ hyp,
    const float* __restrict__ hzp, const float* __restrict__ ax, const float* __restrict__ ay,
    float* __restrict__ pdf) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    pdf[i] = pdf_one(wix[i], wiy[i], wiz[i], hxp[i], hyp[i], hzp[i], ax[i], ay[i]);
}

// Inverse of the cap sampler (Sec. 3.2): the hemisphere normal
// n = M^T h / |M^T h| reflects ws into the cap point c = 2 (n . ws) n - ws
// (reflection law); then 1 - u2 = (c_z + zs) / (1 + zs), i.e.
// u2 = (1 + zs - 2 (n . ws) n_z) / (1 + zs), and u1 = atan2(c_y, c_x) / (2 pi)
// in [0, 1).  Outside the domain both are -1.  The geometry runs in double
// (u2 cancels near the apex of the cap, and c_xy shrinks there), with
// n taken along (hx ay, hy ax, hz ax ay), which needs no division; only the
// azimuth of the double-accurate c is taken in FP32, which keeps its error at
// a few 2^-24 turns however small c_xy is.
__device__ __forceinline__ void inverse_one(float wxf, float wyf, float wzf, float hxf, float hyf,
                                            float hzf, float axf, float ayf, float& u1, float& u2) {
    double e1, e2;
    const double s12 = two_sum((double)wxf * hxf, (double)wyf * hyf, e1);
    const double d0 = two_sum(s12, (double)wzf * hzf, e2) + (e1 + e2);
    const bool ok = (wzf > 0.0f) && (axf > 0.0f) && (ayf > 0.0f) && (hzf > 0.0f) && (d0 > 0.0);
    if (!ok) {
        wxf = 0.0f; wyf = 0.0f; wzf = 1.0f; axf = 1.0f; ayf = 1.0f; hxf = 0.0f; hyf = 0.0f;
        hzf = 1.0f;
    }
    const double ax = axf, ay = ayf, wz = wzf;
    const double px = ax * (double)wxf, py = ay * (double)wyf;
    const double l2 = __builtin_fma(px, px, __builtin_fma(py, py, wz * wz));
    const double il = rsq_f64(l2);
    const double wsx = px * il, wsy = py * il, zs = wz * il;
    const double opz = (l2 * il + wz) * il;  // 1 + zs
    const double mx = (double)hxf * ay, my = (double)hyf * ax, mz = (double)hzf * (ax * ay);
    const double im = rsq_f64(__builtin_fma(mx, mx, __builtin_fma(my, my, mz * mz)));
    const double nx = mx * im, ny = my * im, nz = mz * im;
    const double d2 = 2.0 * __builtin_fma(nx, wsx, __builtin_fma(ny, wsy, nz * zs));
    const double cx = __builtin_fma(d2, nx, -wsx);
    const double cy = __builtin_fma(d2, ny, -wsy);
    const float v2 = (float)(__builtin_fma(-d2, nz, opz) * rcp_f64(opz));
    float t = atan2f((float)cy, (float)cx) * 0.159154943091895336f;
    t = t < 0.0f ? t + 1.0f : t;
    t = t >= 1.0f ? 0.0f : t;
    u1 = ok ? t : -1.0f;
    // a normal at the rim of the cap, rounded to FP32, can map to u2 >= 1:
    // clamp into [0, 1)
    u2 = ok ? fminf(fmaxf(v2, 0.0f), 0x1.fffffep-1f) : -1.0f;
}

template <int G, bool CACHED_OUT, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_inverse_v4(
    int64_t n, const float* __restrict__ wix, const float* __restrict__ wiy,
    const float* __restrict__ wiz, const float* __restrict__ hxp, const float* __restrict__ hyp,
    const float* __restrict__ hzp, const float* __restrict__ ax, const float* __restrict__ ay,
    float* __restrict__ u1p, float* __restrict__ u2p) {
    const int64_t tile = (int64_t)blockIdx.x * BLOCK * 4 * G;
    f4 x[G], y[G], z[G], hx[G], hy[G], hz[G], a[G], b[G];
    load_groups<G, BLOCK, true>(x, wix, tile, n);
    load_groups<G, BLOCK, true>(y, wiy, tile, n);
    load_groups<G, BLOCK, true>(z, wiz, tile, n);
    load_groups<G, BLOCK, true>(hx, hxp, tile, n);
    load_groups<G, BLOCK, true>(hy, hyp, tile, n);
    load_groups<G, BLOCK, true>(hz, hzp, tile, n);
    load_groups<G, BLOCK, true>(a, ax, tile, n);
    load_groups<G, BLOCK, true>(b, ay, tile, n);
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t i0 = group_start<G, BLOCK, true>(tile, g);
        if (i0 + 4 <= n) {
            f4 o1, o2;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float q1, q2;
                inverse_one(x[g][j], y[g][j], z[g][j], hx[g][j], hy[g][j], hz[g][j], a[g][j],
                            b[g][j], q1, q2);
                o1[j] = q1; o2[j] = q2;
            }
            if (CACHED_OUT) store4_cached(u1p + i0, o1); else store4(u1p + i0, o1);
            if (CACHED_OUT) store4_cached(u2p + i0, o2); else store4(u2p + i0, o2);
        } else {
            for (int64_t i = i0; i < n && i < i0 + 4; ++i)
                inverse_one(wix[i], wiy[i], wiz[i], hxp[i], hyp[i], hzp[i], ax[i], ay[i], u1p[i],
                            u2p[i]);
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_inverse_scalar(
    int64_t n, const float* __restrict__ wix, const float* __restrict__ wiy,
    const float* __restrict__ wiz, const float* __restrict__ hxp, const float* __restrict__ hyp,
    const float* __restrict__ hzp, const float* __restrict__ ax, const float* __restrict__ ay,
    float* __restrict__ u1p, float* __restrict__ u2p) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    inverse_one(wix[i], wiy[i], wiz[i], hxp[i], hyp[i], hzp[i], ax[i], ay[i], u1p[i], u2p[i]);
}

__global__ __launch_bounds__(kBlock) void k_uniforms(int64_t n, uint64_t k0, uint32_t tag,
                                                     uint32_t unit, uint32_t key0,
                                                     uint32_t key1, float* __restrict__ u1,
                                                     float* __restrict__ u2) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = k0 + (uint64_t)i;
    const Words w = philox_pair(k >> 1, unit, tag, key0, key1);
    const bool odd = (k & 1u) != 0;
    u1[i] = unit24(odd ? w.w2 : w.w0);
    u2[i] = unit24(odd ? w.w3 : w.w1);
}

__global__ __launch_bounds__(kBlock) void k_philox_blocks(int64_t n,
                                                          const uint32_t* __restrict__ ctr,
                                                          uint32_t key0, uint32_t key1,
                                                          uint32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const Words w = philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3],
                                  key0, key1);
    out[4 * i] = w.w0;
    out[4 * i + 1] = w.w1;
    out[4 * i + 2] = w.w2;
    out[4 * i + 3] = w.w3;
}

// Register-resident sampler benchmark: per lane one view azimuth and
// roughness pair, then `iters` calls with Weyl-sequence uniforms and a view
// elevation that moves each call (so the stretch cannot be hoisted).
template <int METHOD>
__global__ __launch_bounds__(kBlock) void k_microbench(int64_t lanes, int32_t iters,
                                                       uint32_t key0, uint32_t key1,
                                                       uint32_t* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= lanes) return;
    const Words w = philox_pair((uint64_t)t, 0u, 5u, key0, key1);
    float sphi, cphi;
    sincos_turns(unit24(w.w0), &sphi, &cphi);
    // alpha = 10^(-3 U): log-uniform in [1e-3, 1]
    const float ax = __builtin_amdgcn_exp2f(-9.965784284662087f * unit24(w.w1));
    const float ay = __builtin_amdgcn_exp2f(-9.965784284662087f * unit24(w.w2));
    float u1 = unit24(w.w3);
    float u2 = unit24(w.w3 ^ w.w0);
    float mu = unit24(w.w2 ^ w.w1);
    float acc = 0.0f;
    for (int32_t j = 0; j < iters; ++j) {
        u1 += 0.6180339887f;
        u1 -= __builtin_floorf(u1);
        u2 += 0.7548776662f;
        u2 -= __builtin_floorf(u2);
        mu += 0.5698402910f;
        mu -= __builtin_floorf(mu);
        const float cz = __builtin_fmaf(mu, 0.999f, 1e-3f);
        const float sz = fsqrt(__builtin_fmaf(-cz, cz, 1.0f));
        float hx, hy, hz, p;
        sample_one<METHOD, false>(sz * cphi, sz * sphi, cz, ax, ay, u1, u2, hx, hy, hz, p);
        acc += hx + hy + hz;
    }
    out[t] = __float_as_uint(acc);
}

// Bandwidth probe with the sampler's arrays and launch shape.  MODE 0: the
// sampler's traffic (out0 = in0 + in4, out1..3 = in1..3: 20 B read and 16 B
// written per element); MODE 1: the five reads only (a data-dependent store
// that never fires for finite inputs keeps the loads); MODE 2: the four
// writes only (values from the index).
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_stream_probe(
    int64_t n, const float* __restrict__ in0, const float* __restrict__ in1,
    const float* __restrict__ in2, const float* __restrict__ in3,
    const float* __restrict__ in4, float* __restrict__ out0, float* __restrict__ out1,
    float* __restrict__ out2, float* __restrict__ out3) {
    const int64_t tile = (int64_t)blockIdx.x * kTile;
    f4 a[kGroups], b[kGroups], c[kGroups], d[kGroups], e[kGroups];
    if (MODE != 2) {
        load_groups(a, in0, tile, n);
        load_groups(b, in1, tile, n);
        load_groups(c, in2, tile, n);
        load_groups(d, in3, tile, n);
        load_groups(e, in4, tile, n);
    }
#pragma unroll
    for (int g = 0; g < kGroups; ++g) {
        const int64_t i0 = group_start<kGroups>(tile, g);
        if (i0 + 4 <= n) {
            if (MODE == 0) {
                store4(out0 + i0, a[g] + e[g]);
                store4(out1 + i0, b[g]);
                store4(out2 + i0, c[g]);
                store4(out3 + i0, d[g]);
            } else if (MODE == 1) {
                const f4 t = a[g] + b[g] + c[g] + d[g] + e[g];
                const float s4 = t[0] + t[1] + t[2] + t[3];
                if (!(s4 == s4) || s4 == INFINITY) out0[i0] = s4;
            } else {
                const float v = (float)i0;
                store4(out0 + i0, f4{v, v + 1.0f, v + 2.0f, v + 3.0f});
                store4(out1 + i0, f4{v, v, v, v});
                store4(out2 + i0, f4{1.0f, 1.0f, 1.0f, 1.0f});
                store4(out3 + i0, f4{0.0f, 0.0f, 0.0f, 0.0f});
            }
        } else {
            for (int64_t i = i0; i < n && i < i0 + 4; ++i) {
                if (MODE == 0) {
                    out0[i] = in0[i] + in4[i];
                    out1[i] = in1[i];
                    out2[i] = in2[i];
                    out3[i] = in3[i];
                } else if (MODE == 1) {
                    const float s1 = in0[i] + in1[i] + in2[i] + in3[i] + in4[i];
                    if (!(s1 == s1) || s1 == INFINITY) out0[i] = s1;
                } else {
                    out0[i] = (float)i; out1[i] = (float)i; out2[i] = 1.0f; out3[i] = 0.0f;
                }
            }
        }
    }
}


template <int METHOD, bool EU, bool WP>
void launch_sample(bool vec, int64_t n, const float* wix, const float* wiy, const float* wiz,
                   const float* ax, const float* ay, const float* u1, const float* u2,
                   uint64_t index_base, uint32_t k0, uint32_t k1, float* hx, float* hy, float* hz,
                   float* pdf, hipStream_t st) {
    constexpr int G = METHOD == CAPVNDF_CAP_F64 ? kF64Groups : kGroups;
    if (vec) {
        hipLaunchKernelGGL((k_sample_v4<METHOD, EU, WP, G>), dim3(tiles_for<G>(n)),
                           dim3(kBlock), 0, st, n, wix, wiy, wiz, ax, ay, u1, u2, index_base, k0,
                           k1, hx, hy, hz, pdf);
    } else {
        hipLaunchKernelGGL((k_sample_scalar<METHOD, EU, WP>), dim3(grid_for(n)), dim3(kBlock), 0,
                           st, n, wix, wiy, wiz, ax, ay, u1, u2, index_base, k0, k1, hx, hy, hz,
                           pdf);
    }
}

template <int METHOD>
void dispatch_sample(bool vec, bool eu, bool wp, int64_t n, const float* wix, const float* wiy,
                     const float* wiz, const float* ax, const float* ay, const float* u1,
                     const float* u2, uint64_t ib, uint32_t k0, uint32_t k1, float* hx,
                     float* hy, float* hz, float* pdf, hipStream_t st) {
    if (eu && wp)
        launch_sample<METHOD, true, true>(vec, n, wix, wiy, wiz, ax, ay, u1, u2, ib, k0, k1, hx, hy, hz, pdf, st);
    else if (eu)
        launch_sample<METHOD, true, false>(vec, n, wix, wiy, wiz, ax, ay, u1, u2, ib, k0, k1, hx, hy, hz, pdf, st);
    else if (wp)
        launch_sample<METHOD, false, true>(vec, n, wix, wiy, wiz, ax, ay, u1, u2, ib, k0, k1, hx, hy, hz, pdf, st);
    else
        launch_sample<METHOD, false, false>(vec, n, wix, wiy, wiz, ax, ay, u1, u2, ib, k0, k1, hx, hy, hz, pdf, st);
}

}  // namespace
}  // namespace capvndf

using namespace capvndf;

extern "C" int32_t vndf_sample(int64_t n, const float* wix, const float* wiy, const float* wiz,
                               const float* ax, const float* ay, const float* u1, const float* u2,
                               uint64_t seed, uint64_t index_base, int32_t method, float* hx,
                               float* hy, float* hz, float* pdf, void* stream) {
    if (n < 0) return fail(CAPVNDF_ERR_BAD_SIZE, "vndf_sample: n = %lld < 0", (long long)n);
    if (method != CAPVNDF_CAP && method != CAPVNDF_DISK2018 && method != CAPVNDF_CAP_F64)
        return fail(CAPVNDF_ERR_BAD_METHOD, "vndf_sample: unknown method %d", method);
    if ((u1 == nullptr) != (u2 == nullptr))
        return fail(CAPVNDF_ERR_NULL_PTR, "vndf_sample: give both u1 and u2 or neither");
    if (n == 0) return CAPVNDF_OK;
    const void* req[] = {wix, wiy, wiz, ax, ay, hx, hy, hz};
    const char* names[] = {"wix", "wiy", "wiz", "ax", "ay", "hx", "hy", "hz"};
    for (int i = 0; i < 8; ++i)
        if (int32_t rc = check_array(req[i], names[i])) return rc;
    if (u1 != nullptr) {
        if (int32_t rc = check_array(u1, "u1")) return rc;
        if (int32_t rc = check_array(u2, "u2")) return rc;
    }
    if (pdf != nullptr)
        if (int32_t rc = check_array(pdf, "pdf")) return rc;
    bool vec = (index_base % 2) == 0;
    const void* all[] = {wix, wiy, wiz, ax, ay, hx, hy, hz, u1, u2, pdf};
    for (const void* p : all)
        if (p != nullptr && !aligned_to(p, 16)) vec = false;
    const bool eu = u1 != nullptr, wp = pdf != nullptr;
    const hipStream_t st = as_stream(stream);
    for (int64_t o = 0; o < n; o += kSliceElems) {
        const int64_t m = slice_len(n, o);
        const uint64_t ib = index_base + (uint64_t)o;
        if (method == CAPVNDF_CAP)
            dispatch_sample<CAPVNDF_CAP>(vec, eu, wp, m, at(wix, o), at(wiy, o), at(wiz, o),
                                         at(ax, o), at(ay, o), at(u1, o), at(u2, o), ib,
                                         key_lo(seed), key_hi(seed), at(hx, o), at(hy, o),
                                         at(hz, o), at(pdf, o), st);
        else if (method == CAPVNDF_CAP_F64)
            dispatch_sample<CAPVNDF_CAP_F64>(vec, eu, wp, m, at(wix, o), at(wiy, o), at(wiz, o),
                                             at(ax, o), at(ay, o), at(u1, o), at(u2, o), ib,
                                             key_lo(seed), key_hi(seed), at(hx, o), at(hy, o),
                                             at(hz, o), at(pdf, o), st);
        else
            dispatch_sample<CAPVNDF_DISK2018>(vec, eu, wp, m, at(wix, o), at(wiy, o), at(wiz, o),
                                              at(ax, o), at(ay, o), at(u1, o), at(u2, o), ib,
                                              key_lo(seed), key_hi(seed), at(hx, o), at(hy, o),
                                              at(hz, o), at(pdf, o), st);
        if (int32_t rc = check_launch("vndf_sample launch")) return rc;
    }
    return CAPVNDF_OK;
}

extern "C" int32_t vndf_pdf(int64_t n, const float* wix, const float* wiy, const float* wiz,
                            const float* hx, const float* hy, const float* hz, const float* ax,
                            const float* ay, float* pdf, void* stream) {
    if (n < 0) return fail(CAPVNDF_ERR_BAD_SIZE, "vndf_pdf: n = %lld < 0", (long long)n);
    if (n == 0) return CAPVNDF_OK;
    const void* req[] = {wix, wiy, wiz, hx, hy, hz, ax, ay, pdf};
    const char* names[] = {"wix", "wiy", "wiz", "hx", "hy", "hz", "ax", "ay", "pdf"};
    bool vec = true;
    for (int i = 0; i < 9; ++i) {
        if (int32_t rc = check_array(req[i], names[i])) return rc;
        if (!aligned_to(req[i], 16)) vec = false;
    }
    const hipStream_t st = as_stream(stream);
    for (int64_t o = 0; o < n; o += kSliceElems) {
        const int64_t m = slice_len(n, o);
        if (vec)
            hipLaunchKernelGGL((k_pdf_v4<kPdfGroups, kPdfCached, kPdfBlock>),
                               dim3(tiles_for<kPdfGroups, kPdfBlock>(m)), dim3(kPdfBlock), 0, st, m, wix + o, wiy + o, wiz + o, hx + o, hy + o,
                               hz + o, ax + o, ay + o, pdf + o);
        else
            hipLaunchKernelGGL(k_pdf_scalar, dim3(grid_for(m)), dim3(kBlock), 0, st, m, wix + o,
                               wiy + o, wiz + o, hx + o, hy + o, hz + o, ax + o, ay + o, pdf + o);
        if (int32_t rc = check_launch("vndf_pdf launch")) return rc;
    }
    return CAPVNDF_OK;
}

extern "C" int32_t vndf_inverse(int64_t n, const float* wix, const float* wiy, const float* wiz,
                                const float* hx, const float* hy, const float* hz, const float* ax,
                                const float* ay, float* u1, float* u2, void* stream) {
    if (n < 0) return fail(CAPVNDF_ERR_BAD_SIZE, "vndf_inverse: n = %lld < 0", (long long)n);
    if (n == 0) return CAPVNDF_OK;
    const void* req[] = {wix, wiy, wiz, hx, hy, hz, ax, ay, u1, u2};
    const char* names[] = {"wix", "wiy", "wiz", "hx", "hy", "hz", "ax", "ay", "u1", "u2"};
    bool vec = true;
    for (int i = 0; i < 10; ++i) {
        if (int32_t rc = check_array(req[i], names[i])) return rc;
        if (!aligned_to(req[i], 16)) vec = false;
    }
    const hipStream_t st = as_stream(stream);
    for (int64_t o = 0; o < n; o += kSliceElems) {
        const int64_t m = slice_len(n, o);
        if (vec)
            hipLaunchKernelGGL((k_inverse_v4<kInverseGroups, kInverseCached, kInverseBlock>),
                               dim3(tiles_for<kInverseGroups, kInverseBlock>(m)),
                               dim3(kInverseBlock), 0,
                               st, m, wix + o,
                               wiy + o, wiz + o, hx + o, hy + o, hz + o, ax + o, ay + o, u1 + o,
                               u2 + o);
        else
            hipLaunchKernelGGL(k_inverse_scalar, dim3(grid_for(m)), dim3(kBlock), 0, st, m,
                               wix + o, wiy + o, wiz + o, hx + o, hy + o, hz + o, ax + o, ay + o,
                               u1 + o, u2 + o);
        if (int32_t rc = check_launch("vndf_inverse launch")) return rc;
    }
    return CAPVNDF_OK;
}

extern "C" int32_t capvndf_uniforms(uint64_t seed, uint32_t tag, uint32_t unit, uint64_t k0,
                                    int64_t n, float* u1, float* u2, void* stream) {
    if (n < 0) return fail(CAPVNDF_ERR_BAD_SIZE, "capvndf_uniforms: n < 0");
    if (n == 0) return CAPVNDF_OK;
    if (int32_t rc = check_array(u1, "u1")) return rc;
    if (int32_t rc = check_array(u2, "u2")) return rc;
    for (int64_t o = 0; o < n; o += kSliceElems) {
        const int64_t m = slice_len(n, o);
        hipLaunchKernelGGL(k_uniforms, dim3(grid_for(m)), dim3(kBlock), 0, as_stream(stream), m,
                           k0 + (uint64_t)o, tag, unit, key_lo(seed), key_hi(seed), u1 + o, u2 + o);
        if (int32_t rc = check_launch("capvndf_uniforms launch")) return rc;
    }
    return CAPVNDF_OK;
}

extern "C" int32_t capvndf_philox_blocks(int64_t n, const uint32_t* ctr, uint32_t key0,
                                         uint32_t key1, uint32_t* out, void* stream) {
    if (n < 0) return fail(CAPVNDF_ERR_BAD_SIZE, "capvndf_philox_blocks: n < 0");
    if (n == 0) return CAPVNDF_OK;
    if (int32_t rc = check_array(ctr, "ctr")) return rc;
    if (int32_t rc = check_array(out, "out")) return rc;
    for (int64_t o = 0; o < n; o += kSliceElems) {
        const int64_t m = slice_len(n, o);
        hipLaunchKernelGGL(k_philox_blocks, dim3(grid_for(m)), dim3(kBlock), 0, as_stream(stream),
                           m, ctr + 4 * o, key0, key1, out + 4 * o);
        if (int32_t rc = check_launch("capvndf_philox_blocks launch")) return rc;
    }
    return CAPVNDF_OK;
}

extern "C" int32_t vndf_microbench(int32_t method, int64_t lanes, int32_t iters, uint64_t seed,
                                   uint32_t* out, void* stream) {
    if (lanes < 0 || lanes > kSliceElems || iters < 0)
        return fail(CAPVNDF_ERR_BAD_SIZE, "vndf_microbench: lanes must be in [0, 2^31], iters >= 0");
    if (method != CAPVNDF_CAP && method != CAPVNDF_DISK2018 && method != CAPVNDF_CAP_F64)
        return fail(CAPVNDF_ERR_BAD_METHOD, "vndf_microbench: unknown method %d", method);
    if (lanes == 0) return CAPVNDF_OK;
    if (int32_t rc = check_array(out, "out")) return rc;
    const hipStream_t st = as_stream(stream);
    if (method == CAPVNDF_CAP)
        hipLaunchKernelGGL(k_microbench<CAPVNDF_CAP>, dim3(grid_for(lanes)), dim3(kBlock), 0, st,
                           lanes, iters, key_lo(seed), key_hi(seed), out);
    else if (method == CAPVNDF_CAP_F64)
        hipLaunchKernelGGL(k_microbench<CAPVNDF_CAP_F64>, dim3(grid_for(lanes)), dim3(kBlock), 0,
                           st, lanes, iters, key_lo(seed), key_hi(seed), out);
    else
        hipLaunchKernelGGL(k_microbench<CAPVNDF_DISK2018>, dim3(grid_for(lanes)), dim3(kBlock), 0,
                           st, lanes, iters, key_lo(seed), key_hi(seed), out);
    return check_launch("vndf_microbench launch");
}

extern "C" int32_t capvndf_stream_probe(int32_t mode, int64_t n, const float* in0,
                                        const float* in1, const float* in2, const float* in3,
                                        const float* in4, float* out0, float* out1, float* out2,
                                        float* out3, void* stream) {
    if (mode < 0 || mode > 2)
        return fail(CAPVNDF_ERR_BAD_ARG, "capvndf_stream_probe: mode must be 0, 1 or 2");
    if (n < 0) return fail(CAPVNDF_ERR_BAD_SIZE, "capvndf_stream_probe: n < 0");
    if (n == 0) return CAPVNDF_OK;
    const void* req[] = {in0, in1, in2, in3, in4, out0, out1, out2, out3};
    for (const void* p : req) {
        if (int32_t rc = check_array(p, "stream probe array")) return rc;
        if (!aligned_to(p, 16))
            return fail(CAPVNDF_ERR_MISALIGNED, "capvndf_stream_probe: arrays must be 16-byte aligned");
    }
    const hipStream_t st = as_stream(stream);
    for (int64_t o = 0; o < n; o += kSliceElems) {
        const int64_t m = slice_len(n, o);
        const dim3 grid(tiles_for(m)), block(kBlock);
        if (mode == 0)
            hipLaunchKernelGGL(k_stream_probe<0>, grid, block, 0, st, m, in0 + o, in1 + o, in2 + o,
                               in3 + o, in4 + o, out0 + o, out1 + o, out2 + o, out3 + o);
        else if (mode == 1)
            hipLaunchKernelGGL(k_stream_probe<1>, grid, block, 0, st, m, in0 + o, in1 + o, in2 + o,
                               in3 + o, in4 + o, out0 + o, out1 + o, out2 + o, out3 + o);
        else
            hipLaunchKernelGGL(k_stream_probe<2>, grid, block, 0, st, m, in0 + o, in1 + o, in2 + o,
                               in3 + o, in4 + o, out0 + o, out1 + o, out2 + o, out3 + o);
        if (int32_t rc = check_launch("capvndf_stream_probe launch")) return rc;
    }
    return CAPVNDF_OK;
}
