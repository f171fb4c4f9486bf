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

// Reflections within the FP32 path's rounding of the horizon.  The FP32
// normal is within (8 + 48 kappa) 2^-24 of the exact one (first-order count,
// kappa = max(1, ax, ay) / L with L = |M^-T hs|), and wl = 2 (wo.h) h - wo
// multiplies that by 4 and adds the roundings of the dot product, the
// reflection and wo's normalisation: wl_z within (44 + 192 kappa) 2^-24 of 0
// may lie on either side of the horizon, where the weight's slope jumps from
// its live value to 0.  albedo_adj flags such samples (a few in 10^5) with a
// margin >= 0; the adjoint kernels record which lanes had one, and a separate
// pass evaluates them again in double precision, replacing their FP32 terms.
constexpr float kBandC0 = 44.0f * 0x1p-24f;
constexpr float kBandC1 = 192.0f * 0x1p-24f;
// Beyond this conditioning the FP32 sample's terms carry relative errors
// above about 1 % ((35 + 200 kappa) 2^-24); such samples take the double path
// too, wherever their reflection lies.
constexpr float kIllConditioned = 1024.0f;
// the band's width at that conditioning: a sample is flagged if |wl_z| or
// kBandIll is within its band
constexpr float kBandIll = kBandC0 + kBandC1 * kIllConditioned;

// Per-cell (or per-job) constants, uniform across the lanes working on it.
struct CellConst {
    float ox, oy, oz;  // unit view direction
    float ax, ay;
    Stretched s;       // stretched view direction
    float go;          // G1(wo)
    float tgo;         // 2 - G1(wo)
    float tx, ty, tz;  // meridian tangent dwo/dtheta_o
    float rx, ry, rz;  // the view direction as given (for the double-precision path)
    float b1;          // kBandC1 max(1, ax, ay): the horizon band's slope in 1 / L
    bool ok;           // inside the domain
};

__device__ __forceinline__ CellConst cell_setup(float wx, float wy, float wz, float ax, float ay) {
    CellConst c;
    c.ok = (wz > 0.0f) && (ax > 0.0f) && (ay > 0.0f);
    if (!c.ok) {
        wx = 0.0f; wy = 0.0f; wz = 1.0f; ax = 1.0f; ay = 1.0f;
    }
    c.rx = wx;
    c.ry = wy;
    c.rz = wz;
    const float amax = fmaxf(1.0f, fmaxf(ax, ay));
    c.b1 = kBandC1 * amax;
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
// held per lane (uniform values).  For the hardware base-2 exponential each
// lobe keeps b = kappa log2(e) mu and c = kappa log2(e), so that its exponent
// b.w - c is three fused multiply-adds.  The lobe count is a compile-time
// parameter: with a run-time count the compiler evaluated all kMaxLobes lobes
// and selected the live ones.
constexpr int kMaxLobes = 8;

template <int NL>
struct Lobes {
    static constexpr int kN = NL > 0 ? NL : 1;
    float bx[kN], by[kN], bz[kN], nc[kN], lam[kN];  // b, -c, lambda
};

template <int NL>
__device__ __forceinline__ Lobes<NL> load_lobes(const float* __restrict__ p) {
    Lobes<NL> l;
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const float k2 = p[5 * k + 3] * 1.4426950408889634f;
        l.bx[k] = p[5 * k] * k2;
        l.by[k] = p[5 * k + 1] * k2;
        l.bz[k] = p[5 * k + 2] * k2;
        l.nc[k] = -k2;
        l.lam[k] = p[5 * k + 4];
    }
    return l;
}

template <int NL>
__device__ __forceinline__ float lobe_radiance(const Lobes<NL>& l, float wx, float wy, float wz) {
    float r = 0.0f;
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const float e = __builtin_fmaf(l.bx[k], wx, __builtin_fmaf(l.by[k], wy,
                                                                   __builtin_fmaf(l.bz[k], wz, l.nc[k])));
        r = __builtin_fmaf(l.lam[k], __builtin_amdgcn_exp2f(e), r);
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
    float margin;  // >= 0: a flagged sample (see kBandC0), else negative
};

// albedo_adj's value and derivatives in double precision from the cell's
// inputs as given (the same steps; the FP32 view direction, roughness and
// uniforms are exact in double), rounded to FP32 at the end.
__device__ __attribute__((noinline)) AdjTerm albedo_adj_f64(const CellConst& c, float f0f,
                                                            float u1f, float u2f) {
    // cell constants
    const double rx = c.rx, ry = c.ry, rz = c.rz, ax = c.ax, ay = c.ay;
    const double in = rsq_f64(__builtin_fma(rx, rx, __builtin_fma(ry, ry, rz * rz)));
    const double ox = rx * in, oy = ry * in, oz = rz * in;
    const double px = ax * ox, py = ay * oy;
    const double q = __builtin_fma(px, px, py * py);
    const double l2 = __builtin_fma(oz, oz, q);
    const double il = rsq_f64(l2);
    const double lpz = l2 * il + oz;
    const double wsx = px * il, wsy = py * il, zs = oz * il;
    const double opz = lpz * il, omz = q * il * rcp_f64(lpz);
    const double iopz = rcp_f64(opz);
    const double go = 2.0 * zs * iopz, tgo = 2.0 - go;
    const double rho2 = __builtin_fma(ox, ox, oy * oy);
    double tx = oz, ty = 0.0, tz = 0.0;
    if (rho2 > 0.0) {
        const double ir = rsq_f64(rho2);
        tx = oz * ox * ir;
        ty = oz * oy * ir;
        tz = -rho2 * ir;
    }
    // forward sweep
    const double u2 = u2f, a = 1.0 - u2;
    const double hsz = a * opz;
    const double s2 = u2 * opz * (hsz + omz);
    const bool apex = !(s2 > 0.0);
    const double ist = apex ? 0.0 : rsq_f64(s2);
    const double st = s2 * ist;
    double sp, cp;
    sincos_turns_f64(u1f, &sp, &cp);
    const double hsx = __builtin_fma(st, cp, wsx);
    const double hsy = __builtin_fma(st, sp, wsy);
    const double vx = ax * hsx, vy = ay * hsy, vz = hsz;
    const double iL = rsq_f64(__builtin_fma(vx, vx, __builtin_fma(vy, vy, vz * vz)));
    const double hx = vx * iL, hy = vy * iL, hz = vz * iL;
    const double x = __builtin_fma(ox, hx, __builtin_fma(oy, hy, oz * hz));
    const double x2 = x + x;
    const double wlx = __builtin_fma(x2, hx, -ox);
    const double wly = __builtin_fma(x2, hy, -oy);
    const double wlz = __builtin_fma(x2, hz, -oz);
    const double plx = ax * wlx, ply = ay * wly;
    const double pp = __builtin_fma(plx, plx, ply * ply);
    const double m2 = __builtin_fma(wlz, wlz, pp);
    const double im = rsq_f64(m2);
    const double ml = m2 * im;
    const bool live = wlz > 0.0;
    const double wz0 = live ? wlz : 0.0;
    const double iD = rcp_f64(__builtin_fma(go, ml, tgo * wz0));
    const double g = 2.0 * wz0 * iD;
    const double mx = 1.0 - x, mm = mx * mx, m4 = mm * mm;
    const double f0 = f0f, f1 = 1.0 - f0;
    const double F = __builtin_fma(f1, m4 * mx, f0);
    // reverse sweep (as albedo_adj)
    double dx = -5.0 * f1 * m4 * g;
    const double ft2 = F * 2.0 * iD * iD;
    const double e = ft2 * go * im;
    const double dwlz = live ? e * pp : 0.0;
    const double ew = -e * wz0;
    const double dplx = ew * plx, dply = ew * ply;
    const double dgo = -ft2 * wz0 * (ml - wz0);
    double dax = dplx * wlx, day = dply * wly;
    const double dwlx = dplx * ax, dwly = dply * ay;
    dx += 2.0 * __builtin_fma(dwlx, hx, __builtin_fma(dwly, hy, dwlz * hz));
    double dhx = x2 * dwlx, dhy = x2 * dwly, dhz = x2 * dwlz;
    dhx = __builtin_fma(dx, ox, dhx);
    dhy = __builtin_fma(dx, oy, dhy);
    dhz = __builtin_fma(dx, oz, dhz);
    const double dox = __builtin_fma(dx, hx, -dwlx);
    const double doy = __builtin_fma(dx, hy, -dwly);
    const double doz = __builtin_fma(dx, hz, -dwlz);
    const double hd = __builtin_fma(hx, dhx, __builtin_fma(hy, dhy, hz * dhz));
    const double dvx = iL * __builtin_fma(-hx, hd, dhx);
    const double dvy = iL * __builtin_fma(-hy, hd, dhy);
    const double dvz = iL * __builtin_fma(-hz, hd, dhz);
    dax = __builtin_fma(dvx, hsx, dax);
    day = __builtin_fma(dvy, hsy, day);
    const double dhsx = dvx * ax, dhsy = dvy * ay;
    const double dst = __builtin_fma(dhsx, cp, dhsy * sp);
    const double ds2u = apex ? 0.0 : 0.5 * dst * ist * u2;
    const double dopz = __builtin_fma(dvz, a, ds2u * (2.0 * hsz + omz));
    const double domz = ds2u * opz;
    const double dzs = __builtin_fma(dgo * 2.0 * iopz, iopz, dopz - domz);
    AdjTerm r;
    r.w = (float)(F * g);
    r.dax = (float)dax;
    r.day = (float)day;
    r.dth = (float)__builtin_fma(tx, dox, __builtin_fma(ty, doy, tz * doz));
    r.dwsx = (float)dhsx;
    r.dwsy = (float)dhsy;
    r.dzs = (float)dzs;
    r.margin = -1.0f;
    return r;
}

// The adjoint's forward sweep up to the reflected direction (as albedo_fwd,
// keeping the intermediates), and the sample's horizon margin: kappa =
// max(1, ax, ay) iL and band = (44 + 192 kappa) 2^-24; flagged (margin >= 0)
// if |wl_z| <= band or kappa >= kIllConditioned, i.e. band >= kBandIll.
struct Reflected {
    float a, hsz, s2, ist, st, sp, cp, hsx, hsy, iL, hx, hy, hz, x, x2, wlx, wly, wlz, margin;
    bool apex;
};

__device__ __forceinline__ Reflected reflect_sample(const CellConst& c, float u1, float u2) {
    const Stretched& s = c.s;
    Reflected r;
    r.a = 1.0f - u2;
    r.hsz = r.a * s.opz;
    r.s2 = u2 * s.opz * (r.hsz + s.omz);
    // sin(theta_c) = s2 / sqrt(s2), keeping 1 / sin(theta_c) for the reverse
    // sweep; s2 == 0 only at the apex (u2 == 0), where both are taken as 0
    r.apex = !(r.s2 > 0.0f);
    r.ist = rsq(r.s2);
    r.st = r.apex ? 0.0f : r.s2 * r.ist;
    sincos_turns(u1, &r.sp, &r.cp);
    r.hsx = __builtin_fmaf(r.st, r.cp, s.wsx);
    r.hsy = __builtin_fmaf(r.st, r.sp, s.wsy);
    const float vx = c.ax * r.hsx, vy = c.ay * r.hsy, vz = r.hsz;
    r.iL = rsq(__builtin_fmaf(vx, vx, __builtin_fmaf(vy, vy, vz * vz)));
    r.hx = vx * r.iL;
    r.hy = vy * r.iL;
    r.hz = vz * r.iL;
    r.x = __builtin_fmaf(c.ox, r.hx, __builtin_fmaf(c.oy, r.hy, c.oz * r.hz));
    r.x2 = r.x + r.x;
    r.wlx = __builtin_fmaf(r.x2, r.hx, -c.ox);
    r.wly = __builtin_fmaf(r.x2, r.hy, -c.oy);
    r.wlz = __builtin_fmaf(r.x2, r.hz, -c.oz);
    r.margin = __builtin_fmaf(c.b1, r.iL, kBandC0) - fminf(fabsf(r.wlz), kBandIll);
    return r;
}

__device__ __forceinline__ AdjTerm albedo_adj(const CellConst& c, float f0, float u1, float u2) {
    const Stretched& s = c.s;
    // forward sweep
    const Reflected rf = reflect_sample(c, u1, u2);
    const float a = rf.a, hsz = rf.hsz, ist = rf.ist, sp = rf.sp, cp = rf.cp;
    const float hsx = rf.hsx, hsy = rf.hsy, iL = rf.iL, hx = rf.hx, hy = rf.hy, hz = rf.hz;
    const float x = rf.x, x2 = rf.x2, wlx = rf.wlx, wly = rf.wly, wlz = rf.wlz;
    const bool apex = rf.apex;
    const float margin = rf.margin;
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
    r.margin = margin;
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
