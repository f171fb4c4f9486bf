// Per-sample arithmetic of the directional-albedo estimator and its pathwise
// adjoint (device side).
//
// Estimator (Appendix A, "Importance Sampling Using the GGX VNDF", L == 1):
// draw h from the VNDF seen from wo (cap sampler), reflect wo about h
// (wl = 2 (wo.h) h - wo) and weigh by f_r |cos theta_l| / PDF.  With
// PDF = G1(wo) D(h) / (4 cos theta_o) and f_r = F G2 D / (4 cos theta_o
// cos theta_l), D and the cosines cancel: weight = F(wo.h) G2 / G1(wo), and
// for the height-correlated G2 = Go Gl / (Go + Gl - Go Gl) this is
// F Gl / (Go + Gl (1 - Go)).  In the hemisphere space G1(w) = 2 zs / (1 + zs)
// with zs the z of M^-1 w / |M^-1 w|.  Writing Gl this way and multiplying
// through by m = |M^-1 wl| gives the form evaluated here, with one division:
//   g = G2 / G1(wo) = 2 wl_z / (Go m + (2 - Go) wl_z).
#pragma once

#include "device_math.hpp"

namespace capvndf {

// Per-cell (or per-job) constants, uniform across the lanes working on it.
struct CellConst {
    float ox, oy, oz;  // unit view direction
    float ax, ay;
    Stretched s;       // stretched view direction
    float go;          // G1(wo)
    float tgo;         // 2 - G1(wo)
    float tx, ty, tz;  // meridian tangent dwo/dtheta_o
    bool ok;           // inside the domain
};

__device__ __forceinline__ CellConst cell_setup(float wx, float wy, float wz, float ax, float ay) {
    CellConst c;
    c.ok = (wz > 0.0f) && (ax > 0.0f) && (ay > 0.0f);
    if (!c.ok) {
        wx = 0.0f; wy = 0.0f; wz = 1.0f; ax = 1.0f; ay = 1.0f;
    }
    const float in = rsq(__builtin_fmaf(wx, wx, __builtin_fmaf(wy, wy, wz * wz)));
    c.ox = wx * in;
    c.oy = wy * in;
    c.oz = wz * in;
    c.ax = ax;
    c.ay = ay;
    c.s = stretch(c.ox, c.oy, c.oz, ax, ay);
    c.go = 2.0f * c.s.zs * rcp(c.s.opz);
    c.tgo = 2.0f - c.go;
    const float rho2 = __builtin_fmaf(c.ox, c.ox, c.oy * c.oy);
    if (rho2 > 0.0f) {
        const float ir = rsq(rho2);
        c.tx = c.oz * c.ox * ir;
        c.ty = c.oz * c.oy * ir;
        c.tz = -rho2 * ir;
    } else {
        c.tx = c.oz; c.ty = 0.0f; c.tz = 0.0f;
    }
    return c;
}

// Forward term: g = G2/G1 (0 below the horizon) and m5 = (1 - wo.h)^5.
struct FwdTerm {
    float g, m5;
};

__device__ __forceinline__ FwdTerm albedo_fwd(const CellConst& c, float u1, float u2) {
    const CapSample cs = cap_sample(c.s, u1, u2);
    const Normal n = unstretch(cs.hsx, cs.hsy, cs.hsz, c.ax, c.ay);
    const float x = __builtin_fmaf(c.ox, n.hx, __builtin_fmaf(c.oy, n.hy, c.oz * n.hz));
    const float x2 = x + x;
    const float wlx = __builtin_fmaf(x2, n.hx, -c.ox);
    const float wly = __builtin_fmaf(x2, n.hy, -c.oy);
    const float wlz = __builtin_fmaf(x2, n.hz, -c.oz);
    const float plx = c.ax * wlx, ply = c.ay * wly;
    const float m = fsqrt(__builtin_fmaf(plx, plx, __builtin_fmaf(ply, ply, wlz * wlz)));
    // wl_z clamped at 0: g is exactly 0 below the horizon, with a positive
    // denominator (Go m > 0)
    const float wz0 = fmaxf(wlz, 0.0f);
    FwdTerm r;
    r.g = 2.0f * wz0 * rcp(__builtin_fmaf(c.go, m, c.tgo * wz0));
    const float mx = 1.0f - x;
    const float mm = mx * mx;
    r.m5 = mm * mm * mx;
    return r;
}

// Synthetic incident radiance for the direct-illumination estimator: up to
// kMaxLobes spherical-Gaussian lobes L(w) = sum lambda exp(kappa (mu.w - 1)),
// held per lane (uniform values) with kappa pre-scaled by log2(e) for the
// hardware base-2 exponential.  The lobe count is a compile-time parameter:
// with a run-time count the compiler evaluated all kMaxLobes lobes and
// selected the live ones.
constexpr int kMaxLobes = 8;

template <int NL>
struct Lobes {
    static constexpr int kN = NL > 0 ? NL : 1;
    float mx[kN], my[kN], mz[kN], k2[kN], lam[kN];
};

template <int NL>
__device__ __forceinline__ Lobes<NL> load_lobes(const float* __restrict__ p) {
    Lobes<NL> l;
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        l.mx[k] = p[5 * k];
        l.my[k] = p[5 * k + 1];
        l.mz[k] = p[5 * k + 2];
        l.k2[k] = p[5 * k + 3] * 1.4426950408889634f;
        l.lam[k] = p[5 * k + 4];
    }
    return l;
}

template <int NL>
__device__ __forceinline__ float lobe_radiance(const Lobes<NL>& l, float wx, float wy, float wz) {
    float r = 0.0f;
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const float c = __builtin_fmaf(l.mx[k], wx, __builtin_fmaf(l.my[k], wy, l.mz[k] * wz));
        r = __builtin_fmaf(l.lam[k], __builtin_amdgcn_exp2f(__builtin_fmaf(l.k2[k], c, -l.k2[k])), r);
    }
    return r;
}

// Direct-illumination term (Appendix A estimator with radiance L):
// F(wo.h) G2/G1 L(wl), 0 below the horizon.
template <int NL>
__device__ __forceinline__ float radiance_term(const CellConst& c, float f0, const Lobes<NL>& lobes,
                                               float u1, float u2) {
    const CapSample cs = cap_sample(c.s, u1, u2);
    const Normal n = unstretch(cs.hsx, cs.hsy, cs.hsz, c.ax, c.ay);
    const float x = __builtin_fmaf(c.ox, n.hx, __builtin_fmaf(c.oy, n.hy, c.oz * n.hz));
    const float x2 = x + x;
    const float wlx = __builtin_fmaf(x2, n.hx, -c.ox);
    const float wly = __builtin_fmaf(x2, n.hy, -c.oy);
    const float wlz = __builtin_fmaf(x2, n.hz, -c.oz);
    const float plx = c.ax * wlx, ply = c.ay * wly;
    const float m = fsqrt(__builtin_fmaf(plx, plx, __builtin_fmaf(ply, ply, wlz * wlz)));
    const float wz0 = fmaxf(wlz, 0.0f);
    const float g = 2.0f * wz0 * rcp(__builtin_fmaf(c.go, m, c.tgo * wz0));
    const float mx = 1.0f - x;
    const float mm = mx * mx;
    const float F = __builtin_fmaf(1.0f - f0, mm * mm * mx, f0);
    return F * g * lobe_radiance(lobes, wlx, wly, wlz);
}

// Adjoint term for A = mean of w = F g: the weight w and its derivatives at
// fixed (u1, u2).  dax/day/dth hold the direct dependences on alpha and on
// wo (already projected on the meridian tangent); dwsx/dwsy/dzs are the
// adjoints of the stretched view direction ws = (wsx, wsy, zs), whose own
// dependence on (alpha, wo) is the same for every sample of a cell and is
// applied once per thread by ws_chain().
struct AdjTerm {
    float w, dax, day, dth, dwsx, dwsy, dzs;
};

__device__ __forceinline__ AdjTerm albedo_adj(const CellConst& c, float f0, float u1, float u2) {
    const Stretched& s = c.s;
    // forward sweep (as albedo_fwd, keeping the intermediates)
    const float a = 1.0f - u2;
    const float hsz = a * s.opz;
    const float s2 = u2 * s.opz * (hsz + s.omz);
    // sin(theta_c) = s2 / sqrt(s2), keeping 1 / sin(theta_c) for the reverse
    // sweep; s2 == 0 only at the apex (u2 == 0), where both are taken as 0
    const bool apex = !(s2 > 0.0f);
    const float ist = rsq(s2);
    const float st = apex ? 0.0f : s2 * ist;
    float sp, cp;
    sincos_turns(u1, &sp, &cp);
    const float hsx = __builtin_fmaf(st, cp, s.wsx);
    const float hsy = __builtin_fmaf(st, sp, s.wsy);
    const float vx = c.ax * hsx, vy = c.ay * hsy, vz = hsz;
    const float iL = rsq(__builtin_fmaf(vx, vx, __builtin_fmaf(vy, vy, vz * vz)));
    const float hx = vx * iL, hy = vy * iL, hz = vz * iL;
    const float x = __builtin_fmaf(c.ox, hx, __builtin_fmaf(c.oy, hy, c.oz * hz));
    const float x2 = x + x;
    const float wlx = __builtin_fmaf(x2, hx, -c.ox);
    const float wly = __builtin_fmaf(x2, hy, -c.oy);
    const float wlz = __builtin_fmaf(x2, hz, -c.oz);
    const float plx = c.ax * wlx, ply = c.ay * wly;
    const float pp = __builtin_fmaf(plx, plx, ply * ply);
    const float m2 = __builtin_fmaf(wlz, wlz, pp);
    const float im = rsq(m2);
    const float ml = m2 * im;  // |M^-1 wl|
    // wl_z clamped at 0 (see albedo_fwd): below the horizon g and all its
    // derivatives vanish except the direct one in wl_z, which is masked
    const bool live = wlz > 0.0f;
    const float wz0 = fmaxf(wlz, 0.0f);
    const float iD = rcp(__builtin_fmaf(c.go, ml, c.tgo * wz0));
    const float g = 2.0f * wz0 * iD;
    const float mx = 1.0f - x;
    const float mm = mx * mx;
    const float m4 = mm * mm;
    const float f1 = 1.0f - f0;
    const float F = __builtin_fmaf(f1, m4 * mx, f0);

    // reverse sweep, seeded with dw = 1; g = 2 wl_z / D, D = Go m + (2 - Go) wl_z:
    // dg/dwl_z = 2 Go m / D^2, dg/dm = -2 Go wl_z / D^2, dg/dGo = -2 wl_z (m - wl_z) / D^2,
    // and m = |(plx, ply, wl_z)|.
    float dx = -5.0f * f1 * m4 * g;              // through F(x)
    const float ft2 = F * 2.0f * iD * iD;
    const float e = ft2 * c.go * im;             // F dg/dm / m, up to the sign
    const float dwlz = live ? e * pp : 0.0f;     // F (dg/dwl_z + dg/dm wl_z / m)
    const float ew = -e * wz0;
    const float dplx = ew * plx, dply = ew * ply;
    const float dgo = -ft2 * wz0 * (ml - wz0);
    float dax = dplx * wlx;
    float day = dply * wly;
    const float dwlx = dplx * c.ax, dwly = dply * c.ay;
    // wl = 2 x h - wo
    dx += 2.0f * __builtin_fmaf(dwlx, hx, __builtin_fmaf(dwly, hy, dwlz * hz));
    float dhx = x2 * dwlx, dhy = x2 * dwly, dhz = x2 * dwlz;
    // x = wo . h
    dhx = __builtin_fmaf(dx, c.ox, dhx);
    dhy = __builtin_fmaf(dx, c.oy, dhy);
    dhz = __builtin_fmaf(dx, c.oz, dhz);
    const float dox = __builtin_fmaf(dx, hx, -dwlx);
    const float doy = __builtin_fmaf(dx, hy, -dwly);
    const float doz = __builtin_fmaf(dx, hz, -dwlz);
    // h = v / |v|
    const float hd = __builtin_fmaf(hx, dhx, __builtin_fmaf(hy, dhy, hz * dhz));
    const float dvx = iL * __builtin_fmaf(-hx, hd, dhx);
    const float dvy = iL * __builtin_fmaf(-hy, hd, dhy);
    const float dvz = iL * __builtin_fmaf(-hz, hd, dhz);
    // v = (ax hsx, ay hsy, hsz)
    dax = __builtin_fmaf(dvx, hsx, dax);
    day = __builtin_fmaf(dvy, hsy, day);
    const float dhsx = dvx * c.ax, dhsy = dvy * c.ay;
    // hs = (st cos phi + wsx, st sin phi + wsy, (1 - u2)(1 + zs)),
    // st^2 = u2 (1 + zs) ((1 - u2)(1 + zs) + 1 - zs)
    const float dst = __builtin_fmaf(dhsx, cp, dhsy * sp);
    const float ds2u = apex ? 0.0f : 0.5f * dst * ist * u2;
    const float dopz = __builtin_fmaf(dvz, a, ds2u * (2.0f * hsz + s.omz));
    const float domz = ds2u * s.opz;
    const float iopz = rcp(s.opz);
    // Go = 2 zs / (1 + zs), 1 + zs, 1 - zs
    const float dzs = __builtin_fmaf(dgo * 2.0f * iopz, iopz, dopz - domz);

    AdjTerm r;
    r.w = F * g;
    r.dax = dax;
    r.day = day;
    r.dth = __builtin_fmaf(c.tx, dox, __builtin_fmaf(c.ty, doy, c.tz * doz));
    r.dwsx = dhsx;
    r.dwsy = dhsy;
    r.dzs = dzs;
    return r;
}

// Chain the adjoint of ws = p / |p|, p = (ax ox, ay oy, oz), into
// (alpha_x, alpha_y, theta_o): dp = (dws - ws (ws . dws)) / |p|.
__device__ __forceinline__ void ws_chain(const CellConst& c, float dwsx, float dwsy, float dzs,
                                         float& gax, float& gay, float& gth) {
    const Stretched& s = c.s;
    const float wd = __builtin_fmaf(s.wsx, dwsx, __builtin_fmaf(s.wsy, dwsy, s.zs * dzs));
    const float dpx = s.il * __builtin_fmaf(-s.wsx, wd, dwsx);
    const float dpy = s.il * __builtin_fmaf(-s.wsy, wd, dwsy);
    const float dpz = s.il * __builtin_fmaf(-s.zs, wd, dzs);
    gax = __builtin_fmaf(dpx, c.ox, gax);
    gay = __builtin_fmaf(dpy, c.oy, gay);
    gth = __builtin_fmaf(c.tx * c.ax, dpx, __builtin_fmaf(c.ty * c.ay, dpy, __builtin_fmaf(c.tz, dpz, gth)));
}

}  // namespace capvndf
