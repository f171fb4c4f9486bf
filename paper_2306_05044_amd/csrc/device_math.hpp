// Device-side building blocks of the spherical-cap GGX VNDF path (gfx950).
//
// Everything here is per-lane register arithmetic in FP32 (plus 32-bit
// integer work for the random numbers); the kernels in the .hip files wrap it
// with coalesced structure-of-arrays I/O and wavefront/LDS reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace capvndf {

// ---------------------------------------------------------------------------
// Counter-based random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
// SC'11, Sec. 4).  Ten rounds; each multiplies words 0 and 2 by the round
// constants into full 64-bit products and mixes the high halves with the
// other two words and the key; the key advances by the Weyl constants.
// ---------------------------------------------------------------------------
constexpr uint32_t kM0 = 0xD2511F53u;
constexpr uint32_t kM1 = 0xCD9E8D57u;
constexpr uint32_t kW0 = 0x9E3779B9u;
constexpr uint32_t kW1 = 0xBB67AE85u;

// Stream tags of the counter layout: counter = (lo32(k >> 1), unit, tag,
// hi32(k >> 1)), key = (lo32(seed), hi32(seed)); sample k uses words 0,1 when
// k is even and words 2,3 when k is odd.
constexpr uint32_t kTagSample = 2;  // vndf_sample: unit 0, k = index_base + i
constexpr uint32_t kTagAlbedo = 3;  // estimator: unit = cell or job, k = sample

struct Words {
    uint32_t w0, w1, w2, w3;
};

// a ^ b ^ c as one gfx950 three-input logic instruction (truth table 0x96,
// the odd-parity rows; symmetric in its operands).  The compiler does not
// form it from two exclusive-ors by itself, and the round mixes three words.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ Words philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kM0 * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)kM1 * (uint64_t)c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += kW0;
        k1 += kW1;
    }
    return Words{c0, c1, c2, c3};
}

// The block holding samples 2p and 2p+1 of stream (key, tag, unit).
__device__ __forceinline__ Words philox_pair(uint64_t p, uint32_t unit, uint32_t tag,
                                             uint32_t key0, uint32_t key1) {
    return philox4x32_10((uint32_t)p, unit, tag, (uint32_t)(p >> 32), key0, key1);
}

// Top 24 bits of a word as a float in [0, 1): exact, and 1 - u is exact too.
__device__ __forceinline__ float unit24(uint32_t w) { return (float)(w >> 8) * 0x1p-24f; }

// ---------------------------------------------------------------------------
// sin(2 pi u) and cos(2 pi u) for the azimuth.  The hardware sine and cosine
// take their argument in turns (revolutions), so the azimuth needs no
// multiplication by 2 pi and no range reduction for u in [0, 1).  Measured on
// gfx950 over every point of the 2^-24 lattice in [0, 1): absolute error at
// most 1.25e-7 (about two ulps of 1), far inside the sampler's tolerance.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sincos_turns(float u, float* s, float* c) {
    *s = __builtin_amdgcn_sinf(u);
    *c = __builtin_amdgcn_cosf(u);
}

// Hardware reciprocal, reciprocal square root and square root (about 1 ulp).
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

constexpr float kInvPi = 0.318309886183790671538f;

// ---------------------------------------------------------------------------
// Step 1 of the general sampler: warp wi by M^-1 = diag(ax, ay, 1) and
// normalise.  Besides ws = (wsx, wsy, zs) this keeps 1 + zs and 1 - zs in
// cancellation-free forms: with q = (ax wx)^2 + (ay wy)^2 and l = |M^-1 wi|,
// 1 + zs = (l + wz) / l and 1 - zs = q / (l (l + wz)).
// ---------------------------------------------------------------------------
struct Stretched {
    float wsx, wsy, zs;
    float opz;  // 1 + zs
    float omz;  // 1 - zs
    float il;   // 1 / l
};

__device__ __forceinline__ Stretched stretch(float wx, float wy, float wz, float ax, float ay) {
    const float px = ax * wx;
    const float py = ay * wy;
    const float q = __builtin_fmaf(px, px, py * py);
    const float l2 = __builtin_fmaf(wz, wz, q);
    const float il = rsq(l2);
    const float l = l2 * il;
    const float lpz = l + wz;
    Stretched s;
    s.wsx = px * il;
    s.wsy = py * il;
    s.zs = wz * il;
    s.opz = lpz * il;
    s.omz = q * il * rcp(lpz);
    s.il = il;
    return s;
}

// ---------------------------------------------------------------------------
// Step 2 with the spherical cap (Sec. 3.3): c uniform on the cap z in
// (-zs, 1] (u2 = 0 at the apex, azimuth 2 pi u1), half vector hs = c + ws,
// left unnormalised.  The cap height z = (1 - u2)(1 + zs) - zs enters only
// through z + zs = (1 - u2)(1 + zs) and 1 - z^2 = u2 (1 + zs) (z + zs + 1 - zs),
// which avoids the cancellations of forming z and 1 - z^2 directly.
// ---------------------------------------------------------------------------
struct CapSample {
    float hsx, hsy, hsz;  // unnormalised half vector in the hemisphere space
    float st, cp, sp;     // sin(theta_c), cos(phi), sin(phi)
};

__device__ __forceinline__ CapSample cap_sample(const Stretched& s, float u1, float u2) {
    CapSample r;
    const float a = 1.0f - u2;
    r.hsz = a * s.opz;
    const float s2 = u2 * s.opz * (r.hsz + s.omz);
    r.st = fsqrt(s2);
    sincos_turns(u1, &r.sp, &r.cp);
    r.hsx = __builtin_fmaf(r.st, r.cp, s.wsx);
    r.hsy = __builtin_fmaf(r.st, r.sp, s.wsy);
    return r;
}

// ---------------------------------------------------------------------------
// Step 3: warp the normal back with M^-T = diag(ax, ay, 1) and normalise.
// The VNDF pdf at that normal follows from Eq. (1) in the hemisphere space:
// M^T h = hs / L with L = |M^-T hs|, ws . hs_n = |hs| / 2 (since |c| = |ws| =
// 1), so pdf = L^3 / (pi ax ay (1 + zs) |hs|^2).  It equals
// G1(wi) max(0, wi.h) D(h) / wz.
// ---------------------------------------------------------------------------
struct Normal {
    float hx, hy, hz;
    float vx, vy, vz;  // M^-T hs
    float iL;          // 1 / |M^-T hs|
};

__device__ __forceinline__ Normal unstretch(float hsx, float hsy, float hsz, float ax, float ay) {
    Normal n;
    n.vx = ax * hsx;
    n.vy = ay * hsy;
    n.vz = hsz;
    const float L2 = __builtin_fmaf(n.vx, n.vx, __builtin_fmaf(n.vy, n.vy, n.vz * n.vz));
    n.iL = rsq(L2);
    n.hx = n.vx * n.iL;
    n.hy = n.vy * n.iL;
    n.hz = n.vz * n.iL;
    return n;
}

__device__ __forceinline__ float cap_pdf(const Stretched& s, const CapSample& c, const Normal& n,
                                         float ax, float ay) {
    const float L2 = __builtin_fmaf(n.vx, n.vx, __builtin_fmaf(n.vy, n.vy, n.vz * n.vz));
    const float hs2 = __builtin_fmaf(c.hsx, c.hsx, __builtin_fmaf(c.hsy, c.hsy, c.hsz * c.hsz));
    const float L3 = L2 * L2 * n.iL;
    return L3 * kInvPi * rcp(ax * ay * s.opz * hs2);
}

// The same cap sample and pdf evaluated in double precision from the FP32
// inputs and uniforms, rounded to FP32 only at the end.  The FP32 evaluation
// above forms the half vector hs = c + ws from unit vectors, so its absolute
// rounding of O(2^-24) reaches h and the pdf relatively as
// O(2^-24 (1 + max(ax, ay) / L + 1 / |hs|)), which exceeds 2e-6 on a few
// samples in 10^4 of a log-uniform roughness workload (near-grazing halves).
// In double the same steps leave O(2^-50) times that factor.  The double
// arithmetic is kept to what that needs: reciprocals and reciprocal square
// roots from the hardware estimates refined by a Newton step (which squares
// the relative error), and sin/cos(2 pi u1) by an exact
// quadrant reduction (u1 has 24 fraction bits) and Taylor polynomials on
// [-pi/4, pi/4] whose truncation error is below 1e-18.
constexpr double kPiD = 3.14159265358979323846;
constexpr double kHalfPiD = 1.57079632679489661923;

// The hardware double estimates are good to 2^-24.2 relative (measured on
// gfx950 over 2^24 random doubles with exponents -60..60); one Newton step
// squares that to about 2^-48, ample for results rounded to FP32 even where
// the sampler's conditioning reaches 10^7.
__device__ __forceinline__ double rcp_f64(double x) {
    const double y = __builtin_amdgcn_rcp(x);
    return y * __builtin_fma(-x, y, 2.0);
}

__device__ __forceinline__ double rsq_f64(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    return y * __builtin_fma(-0.5 * x * y, y, 1.5);
}

__device__ __forceinline__ void sincos_turns_f64(float u, double* sn, double* cs) {
    const double v = 4.0 * (double)u;  // exact
    const double k = __builtin_rint(v);
    const double x = (v - k) * kHalfPiD;  // v - k exact, |x| <= pi/4
    const double x2 = x * x;
    // sin x = x (1 - x^2/3! + x^4/5! - ... - x^16/17!), cos x = 1 - x^2/2! + ... + x^16/16!
    double ps = 1.0 / 355687428096000.0;
    ps = __builtin_fma(ps, x2, -1.0 / 1307674368000.0);
    ps = __builtin_fma(ps, x2, 1.0 / 6227020800.0);
    ps = __builtin_fma(ps, x2, -1.0 / 39916800.0);
    ps = __builtin_fma(ps, x2, 1.0 / 362880.0);
    ps = __builtin_fma(ps, x2, -1.0 / 5040.0);
    ps = __builtin_fma(ps, x2, 1.0 / 120.0);
    ps = __builtin_fma(ps, x2, -1.0 / 6.0);
    const double sx = __builtin_fma(ps * x2, x, x);
    double pc = 1.0 / 20922789888000.0;
    pc = __builtin_fma(pc, x2, -1.0 / 87178291200.0);
    pc = __builtin_fma(pc, x2, 1.0 / 479001600.0);
    pc = __builtin_fma(pc, x2, -1.0 / 3628800.0);
    pc = __builtin_fma(pc, x2, 1.0 / 40320.0);
    pc = __builtin_fma(pc, x2, -1.0 / 720.0);
    pc = __builtin_fma(pc, x2, 1.0 / 24.0);
    pc = __builtin_fma(pc, x2, -0.5);
    const double cx = __builtin_fma(pc, x2, 1.0);
    // the angle is (k + x / (pi/2)) quarter turns
    const int q = (int)k & 3;
    const double s1 = (q & 1) ? cx : sx;
    const double c1 = (q & 1) ? sx : cx;
    *sn = (q & 2) ? -s1 : s1;
    *cs = ((q + 1) & 2) ? -c1 : c1;
}

template <bool WITH_PDF>
__device__ __forceinline__ void cap_sample_f64(float wxf, float wyf, float wzf, float axf,
                                               float ayf, float u1f, float u2f, float& hx,
                                               float& hy, float& hz, float& pdf) {
    const double wz = wzf, ax = axf, ay = ayf;
    const double px = ax * (double)wxf, py = ay * (double)wyf;
    const double q = __builtin_fma(px, px, py * py);
    const double l2 = __builtin_fma(wz, wz, q);
    const double il = rsq_f64(l2);
    const double l = l2 * il;
    const double lpz = l + wz;
    const double opz = lpz * il;                // 1 + zs
    const double omz = q * il * rcp_f64(lpz);   // 1 - zs
    const double u2 = u2f;
    const double hsz = (1.0 - u2) * opz;        // z + zs
    const double s2 = u2 * opz * (hsz + omz);   // sin^2 of the cap angle
    const double st = s2 > 0.0 ? s2 * rsq_f64(s2) : 0.0;
    double sp, cp;
    sincos_turns_f64(u1f, &sp, &cp);
    const double hsx = __builtin_fma(st, cp, px * il);
    const double hsy = __builtin_fma(st, sp, py * il);
    const double vx = ax * hsx, vy = ay * hsy;
    const double L2 = __builtin_fma(vx, vx, __builtin_fma(vy, vy, hsz * hsz));
    const double iL = rsq_f64(L2);
    hx = (float)(vx * iL);
    hy = (float)(vy * iL);
    hz = (float)(hsz * iL);
    if (WITH_PDF) {
        const double hs2 = __builtin_fma(hsx, hsx, __builtin_fma(hsy, hsy, hsz * hsz));
        pdf = (float)(L2 * L2 * iL * rcp_f64(kPiD * ax * ay * opz * hs2));
    }
}

// Heitz's 2018 cross-section sampler (Sec. 2), the comparison baseline, in the
// hemisphere space: orthonormal basis around ws, polar disk sample, warp of
// the second coordinate by s = (1 + zs) / 2, reprojection.  Returns the unit
// hemisphere normal and its height ti above the disk (ws . wm = ti).
struct DiskSample {
    float mx, my, mz, ti;
};

__device__ __forceinline__ DiskSample disk2018_sample(const Stretched& s, float u1, float u2) {
    const float tmp = __builtin_fmaf(s.wsx, s.wsx, s.wsy * s.wsy);
    float w1x = 1.0f, w1y = 0.0f;
    if (tmp > 0.0f) {
        const float it = rsq(tmp);
        w1x = -s.wsy * it;
        w1y = s.wsx * it;
    }
    // w2 = ws x w1 with w1 = (w1x, w1y, 0)
    const float w2x = -s.zs * w1y;
    const float w2y = s.zs * w1x;
    const float w2z = __builtin_fmaf(s.wsx, w1y, -s.wsy * w1x);
    float sp, cp;
    sincos_turns(u1, &sp, &cp);
    const float r = fsqrt(u2);
    const float t1 = r * cp;
    float t2 = r * sp;
    const float hs = 0.5f * s.opz;
    const float omt = 1.0f - t1 * t1;
    t2 = __builtin_fmaf(0.5f * s.omz, fsqrt(omt), hs * t2);
    const float ti = fsqrt(fmaxf(omt - t2 * t2, 0.0f));
    DiskSample d;
    d.mx = __builtin_fmaf(t1, w1x, __builtin_fmaf(t2, w2x, ti * s.wsx));
    d.my = __builtin_fmaf(t1, w1y, __builtin_fmaf(t2, w2y, ti * s.wsy));
    d.mz = __builtin_fmaf(t2, w2z, ti * s.zs);
    d.ti = ti;
    return d;
}

// pdf of a unit hemisphere normal m seen from ws, at h = M^-T m / |M^-T m|:
// (ws . m) / (pi (1 + zs) / 2) * L^3 / (ax ay), L = |M^-T m|.
__device__ __forceinline__ float disk_pdf(const Stretched& s, const DiskSample& d,
                                          const Normal& n, float ax, float ay) {
    const float L2 = __builtin_fmaf(n.vx, n.vx, __builtin_fmaf(n.vy, n.vy, n.vz * n.vz));
    const float L3 = L2 * L2 * n.iL;
    const float dot = __builtin_fmaf(s.wsx, d.mx, __builtin_fmaf(s.wsy, d.my, s.zs * d.mz));
    return fmaxf(dot, 0.0f) * 2.0f * kInvPi * L3 * rcp(ax * ay * s.opz);
}

// ---------------------------------------------------------------------------
// Compensated accumulation.  Knuth's TwoSum folds an addend into (s, c) with
// the rounding error of every addition kept in c; merge() combines two such
// pairs (used across lanes, waves and blocks in a fixed order).
// ---------------------------------------------------------------------------
struct Comp {
    float s, c;
};

__device__ __forceinline__ void comp_add(Comp& a, float x) {
    const float t = a.s + x;
    const float bp = t - a.s;
    const float ap = t - bp;
    a.c += (a.s - ap) + (x - bp);
    a.s = t;
}

__device__ __forceinline__ Comp comp_merge(const Comp& a, const Comp& b) {
    Comp r;
    const float t = a.s + b.s;
    const float bp = t - a.s;
    const float ap = t - bp;
    r.c = (a.c + b.c) + ((a.s - ap) + (b.s - bp));
    r.s = t;
    return r;
}

}  // namespace capvndf
