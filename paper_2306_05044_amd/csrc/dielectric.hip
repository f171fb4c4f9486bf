// Rough-dielectric (reflection + transmission) sampling with the spherical-cap
// VNDF, and the density of that sampler at given directions.
//
// The paper applies its sampler unchanged to rough dielectrics and takes the
// transmission model from Walter, Marschner, Li and Torrance, "Microfacet
// models for refraction through rough surfaces" (EGSR 2007): a visible normal
// h is drawn from the VNDF seen from wi (Sec. 3.3 here), the lobe is chosen
// with probability F (Fresnel reflectance at wi . h), and wi is reflected or
// refracted about h.  wi lies on the upper side; eta = n_lower / n_upper.
//
// Streaming layout as for the VNDF sampler: structure of arrays, 20 B read
// and 20 B written per tuple (wo, pdf, weight), 16-byte non-temporal accesses.
#include "common.hpp"
#include "device_math.hpp"
#include "stream_io.hpp"

namespace capvndf {
namespace {

// vec4 groups per lane: the sampler draws a whole Philox block per tuple and
// the pdf kernel reads eight arrays, so both keep fewer loads in flight per
// lane than the VNDF sampler and run more waves (measured: 2 and 1 groups
// beat 4 by 3-4 %); the pdf kernel's small output goes through the cache
// (3 % faster than a non-temporal store).
constexpr int kSampleGroups = 2;
constexpr int kSampleBlock = 256;  // 3 % faster than 128 threads for this kernel
#ifndef CAPVNDF_DIELECTRIC_PDF_GROUPS
#define CAPVNDF_DIELECTRIC_PDF_GROUPS 1
#endif
constexpr int kPdfGroups = CAPVNDF_DIELECTRIC_PDF_GROUPS;
constexpr int kPdfBlock = 128;  // 256 threads: 4 % slower for this kernel

// Random numbers of the dielectric sampler: one Philox block per tuple,
// counter (lo32(k), 0, 5, hi32(k)) with k = index_base + i, key (lo32(seed),
// hi32(seed)); u1, u2, u3 from words 0, 1, 2.
constexpr uint32_t kTagDielectric = 5;

struct Eta {
    float eta, eta2, eta2m1, ieta;  // eta, eta^2, eta^2 - 1, 1 / eta (rounded from double)
};

// Unpolarised Fresnel reflectance at cos_i = c > 0 with g = eta cos_t =
// sqrt(eta^2 - 1 + c^2) (Snell's law): r_s = (c - g) / (c + g), r_p =
// (eta^2 c - g) / (eta^2 c + g), F = (r_s^2 + r_p^2) / 2; F = 1 when g^2 <= 0
// (total internal reflection).  Returns F and g (0 under total reflection).
__device__ __forceinline__ float fresnel(float c, const Eta& e, float& g) {
    const float g2 = __builtin_fmaf(c, c, e.eta2m1);
    g = fsqrt(fmaxf(g2, 0.0f));
    const float rs = (c - g) * rcp(c + g);
    const float ec = e.eta2 * c;
    const float rp = (ec - g) * rcp(ec + g);
    const float f = 0.5f * __builtin_fmaf(rs, rs, rp * rp);
    return g2 > 0.0f ? f : 1.0f;
}

struct DielectricOut {
    float wox, woy, woz, pdf, weight;
};

// One tuple.  With hs the cap sample's half vector (hemisphere space),
// L = |M^-T hs| and l = |M^-1 wi|:
//   c = wi . h = l |hs|^2 / (2 L)      (ws . hs = |hs|^2 / 2, no dot product),
//   reflection    wo = 2 c h - wi,                 pdf = F p_h / (4 c),
//   transmission  wo = ((c - g) h - wi) / eta,      pdf = (1 - F) p_h eta g / (c - g)^2,
// where p_h is the fused VNDF pdf at h and the transmission Jacobian
// eta^2 |wo.h| / (wi.h + eta wo.h)^2 used wo . h = -g / eta.  The weight
// f |wo.n| / pdf is G2 / G1(wi) = (1 + L_i) / (1 + L_i + L_o) for both lobes,
// = |wo_z| (1 + z_i) / (z_i l_o + |wo_z|) with z_i = w_z / l and
// l_o = |M^-1 wo|.  A direction on the wrong side for its lobe is no sample
// (pdf and weight 0); inputs outside the domain give wo = (0, 0, 1) and 0.
__device__ __forceinline__ DielectricOut dielectric_one(float wx, float wy, float wz, float ax,
                                                        float ay, float u1, float u2, float u3,
                                                        const Eta& e) {
    const bool ok = (wz > 0.0f) && (ax > 0.0f) && (ay > 0.0f);
    if (!ok) {
        wx = 0.0f; wy = 0.0f; wz = 1.0f; ax = 1.0f; ay = 1.0f;
    }
    const Stretched s = stretch(wx, wy, wz, ax, ay);
    const CapSample cs = cap_sample(s, u1, u2);
    const Normal n = unstretch(cs.hsx, cs.hsy, cs.hsz, ax, ay);
    const float ph = cap_pdf(s, cs, n, ax, ay);
    const float hs2 =
        __builtin_fmaf(cs.hsx, cs.hsx, __builtin_fmaf(cs.hsy, cs.hsy, cs.hsz * cs.hsz));
    const float c = 0.5f * hs2 * n.iL * rcp(s.il);
    float g;
    const float f = fresnel(c, e, g);
    const bool refl = u3 < f;
    // reflection: wo = a h - b wi with a = 2c, b = 1; transmission a = (c - g)/eta, b = 1/eta
    const float a = refl ? 2.0f * c : (c - g) * e.ieta;
    const float b = refl ? 1.0f : e.ieta;
    DielectricOut o;
    o.wox = __builtin_fmaf(a, n.hx, -b * wx);
    o.woy = __builtin_fmaf(a, n.hy, -b * wy);
    o.woz = __builtin_fmaf(a, n.hz, -b * wz);
    const float cg = c - g;
    const float pdf = refl ? f * ph * rcp(4.0f * c) : (1.0f - f) * ph * e.eta * g * rcp(cg * cg);
    const float qx = ax * o.wox, qy = ay * o.woy;
    const float azo = fabsf(o.woz);
    const float lo = fsqrt(__builtin_fmaf(qx, qx, __builtin_fmaf(qy, qy, o.woz * o.woz)));
    const float w = azo * s.opz * rcp(__builtin_fmaf(s.zs, lo, azo));
    const bool valid = ok && (refl ? o.woz > 0.0f : o.woz < 0.0f);
    o.pdf = valid ? pdf : 0.0f;
    o.weight = valid ? w : 0.0f;
    if (!ok) {
        o.wox = 0.0f; o.woy = 0.0f; o.woz = 1.0f;
    }
    return o;
}

__device__ __forceinline__ void dielectric_u(uint64_t k, uint32_t key0, uint32_t key1, float& u1,
                                             float& u2, float& u3) {
    const Words w = philox4x32_10((uint32_t)k, 0u, kTagDielectric, (uint32_t)(k >> 32), key0, key1);
    u1 = unit24(w.w0);
    u2 = unit24(w.w1);
    u3 = unit24(w.w2);
}

// Vector path (arrays 16-byte aligned): tiles of BLOCK * 4 * G tuples, all
// loads of a lane issued before any arithmetic.
template <int G, int BLOCK, bool EXPLICIT_U>
__global__ __launch_bounds__(BLOCK) void k_dielectric_v4(
    int64_t n, const float* __restrict__ wix, const float* __restrict__ wiy,
    const float* __restrict__ wiz, const float* __restrict__ ax, const float* __restrict__ ay,
    const float* __restrict__ u1p, const float* __restrict__ u2p, const float* __restrict__ u3p,
    Eta e, uint64_t index_base, uint32_t key0, uint32_t key1, float* __restrict__ wox,
    float* __restrict__ woy, float* __restrict__ woz, float* __restrict__ pdf,
    float* __restrict__ weight) {
    const int64_t tile = (int64_t)blockIdx.x * BLOCK * 4 * G;
    f4 x[G], y[G], z[G], a[G], b[G], r1[G], r2[G], r3[G];
    load_groups<G, BLOCK>(x, wix, tile, n);
    load_groups<G, BLOCK>(y, wiy, tile, n);
    load_groups<G, BLOCK>(z, wiz, tile, n);
    load_groups<G, BLOCK>(a, ax, tile, n);
    load_groups<G, BLOCK>(b, ay, tile, n);
    if (EXPLICIT_U) {
        load_groups<G, BLOCK>(r1, u1p, tile, n);
        load_groups<G, BLOCK>(r2, u2p, tile, n);
        load_groups<G, BLOCK>(r3, u3p, tile, n);
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t i0 = group_start<G, BLOCK>(tile, g);
        if (i0 + 4 <= n) {
            f4 ox, oy, oz, op, ow;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float u1, u2, u3;
                if (EXPLICIT_U) {
                    u1 = r1[g][j]; u2 = r2[g][j]; u3 = r3[g][j];
                } else {
                    dielectric_u(index_base + (uint64_t)(i0 + j), key0, key1, u1, u2, u3);
                }
                const DielectricOut o =
                    dielectric_one(x[g][j], y[g][j], z[g][j], a[g][j], b[g][j], u1, u2, u3, e);
                ox[j] = o.wox; oy[j] = o.woy; oz[j] = o.woz; op[j] = o.pdf; ow[j] = o.weight;
            }
            store4(wox + i0, ox);
            store4(woy + i0, oy);
            store4(woz + i0, oz);
            store4(pdf + i0, op);
            store4(weight + i0, ow);
        } else {
            for (int64_t i = i0; i < n && i < i0 + 4; ++i) {
                float u1, u2, u3;
                if (EXPLICIT_U) {
                    u1 = u1p[i]; u2 = u2p[i]; u3 = u3p[i];
                } else {
                    dielectric_u(index_base + (uint64_t)i, key0, key1, u1, u2, u3);
                }
                const DielectricOut o = dielectric_one(wix[i], wiy[i], wiz[i], ax[i], ay[i], u1, u2, u3, e);
                wox[i] = o.wox; woy[i] = o.woy; woz[i] = o.woz; pdf[i] = o.pdf; weight[i] = o.weight;
            }
        }
    }
}

// Scalar path (any 4-byte alignment): one tuple per lane.
template <bool EXPLICIT_U>
__global__ __launch_bounds__(kBlock) void k_dielectric_scalar(
    int64_t n, const float* __restrict__ wix, const float* __restrict__ wiy,
    const float* __restrict__ wiz, const float* __restrict__ ax, const float* __restrict__ ay,
    const float* __restrict__ u1p, const float* __restrict__ u2p, const float* __restrict__ u3p,
    Eta e, uint64_t index_base, uint32_t key0, uint32_t key1, float* __restrict__ wox,
    float* __restrict__ woy, float* __restrict__ woz, float* __restrict__ pdf,
    float* __restrict__ weight) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    float u1, u2, u3;
    if (EXPLICIT_U) {
        u1 = u1p[i]; u2 = u2p[i]; u3 = u3p[i];
    } else {
        dielectric_u(index_base + (uint64_t)i, key0, key1, u1, u2, u3);
    }
    const DielectricOut o = dielectric_one(wix[i], wiy[i], wiz[i], ax[i], ay[i], u1, u2, u3, e);
    wox[i] = o.wox; woy[i] = o.woy; woz[i] = o.woz; pdf[i] = o.pdf; weight[i] = o.weight;
}

// Density of the sampler at a given unit pair (wi, wo).  The half vector is
// t = wi + wo (wo above: reflection) or t = -(wi + eta wo) (wo below:
// transmission), h = t / |t| turned to the upper side.  With the VNDF of
// Eq. (1) written as p_h = 2 (wi.h) / ((l + w_z) pi ax ay k^2), k = |M^T h|^2:
//   reflection    pdf = F p_h / (4 |wo.h|) = F (wi.h / |wo.h|) / (2 (l + w_z) pi ax ay k^2),
//   transmission  pdf = (1 - F) p_h eta^2 |wo.h| / |t|^2,
// since (wi.h + eta wo.h)^2 = |t|^2 for any lengths of wi and wo.  For exactly
// unit vectors wi.h = wo.h in reflection; FP32 inputs are unit only up to
// rounding, which moves wi.h - wo.h by about 1e-7 / |t|, so the ratio is kept
// and the density is the one of the definition at the given vectors.  Zero
// unless wi.h > 0 (and wo.h > 0 for reflection, wo.h < 0 for transmission),
// outside the domain, and for wo_z = 0.
//
// Evaluated in double precision:
// the half vector t = +-(wi + k wo) (k = 1 reflection, eta transmission), the
// cosines wi.h and wo.h and the Fresnel terms all cancel in FP32 near grazing
// angles, the critical angle or wo ~ -wi; in double the same steps keep the
// result at the FP32 rounding of the exact density up to a few ulps.  M^T h
// is taken along (hx ay, hy ax, hz ax ay) to avoid divisions.  The kernel is
// bound by HBM traffic, which hides the double arithmetic.
__device__ __forceinline__ float dielectric_pdf_one(float wxf, float wyf, float wzf, float oxf,
                                                    float oyf, float ozf, float axf, float ayf,
                                                    const Eta& e) {
    const bool ok0 = (wzf > 0.0f) && (axf > 0.0f) && (ayf > 0.0f) && (ozf != 0.0f);
    if (!ok0) {
        wxf = 0.0f; wyf = 0.0f; wzf = 1.0f; axf = 1.0f; ayf = 1.0f; oxf = 0.0f; oyf = 0.0f;
        ozf = 1.0f;
    }
    const double wx = wxf, wy = wyf, wz = wzf, ox = oxf, oy = oyf, oz = ozf;
    const double ax = axf, ay = ayf;
    const bool refl = ozf > 0.0f;
    const double eta = e.eta;
    const double k = refl ? 1.0 : eta;
    const double sgn = refl ? 1.0 : -1.0;
    const double tx = sgn * __builtin_fma(k, ox, wx);
    const double ty = sgn * __builtin_fma(k, oy, wy);
    const double tz = sgn * __builtin_fma(k, oz, wz);
    const double t2 = __builtin_fma(tx, tx, __builtin_fma(ty, ty, tz * tz));
    const double it = __builtin_copysign(rsq_f64(t2), tz);
    const double hx = tx * it, hy = ty * it, hz = tz * it;
    const double ci = __builtin_fma(wx, hx, __builtin_fma(wy, hy, wz * hz));
    const double co = __builtin_fma(ox, hx, __builtin_fma(oy, hy, oz * hz));
    // Fresnel (as fresnel() above) with g = sqrt(eta^2 - 1 + ci^2)
    const double g2 = __builtin_fma(ci, ci, __builtin_fma(eta, eta, -1.0));
    const double g = g2 > 0.0 ? g2 * rsq_f64(g2) : 0.0;
    const double rs = (ci - g) * rcp_f64(ci + g);
    const double ec = eta * eta * ci;
    const double rp = (ec - g) * rcp_f64(ec + g);
    const double f = g2 > 0.0 ? 0.5 * __builtin_fma(rs, rs, rp * rp) : 1.0;
    const double px = ax * wx, py = ay * wy;
    const double l2 = __builtin_fma(px, px, __builtin_fma(py, py, wz * wz));
    const double l = l2 * rsq_f64(l2);
    const double axy = ax * ay;
    const double kx = hx * ay, ky = hy * ax, kz = hz * axy;
    const double K = __builtin_fma(kx, kx, __builtin_fma(ky, ky, kz * kz));
    // the VNDF density at h (Eq. (1)) times 1 / (2 ci): pi ax ay k^2 = pi K^2 / (ax ay)^3
    const double base = (axy * axy * axy) * rcp_f64((l + wz) * kPiD * K * K);
    const bool side = refl ? co > 0.0 : co < 0.0;
    const double p = refl ? 0.5 * f * base * ci * rcp_f64(side ? co : 1.0)
                          : (1.0 - f) * 2.0 * ci * base * (eta * eta) * __builtin_fabs(co) *
                                rcp_f64(t2);
    const bool valid = ok0 && ci > 0.0 && hz > 0.0 && side;
    return valid ? (float)p : 0.0f;
}

template <int G, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_dielectric_pdf_v4(
    int64_t n, const float* __restrict__ wix, const float* __restrict__ wiy,
    const float* __restrict__ wiz, const float* __restrict__ woxp, const float* __restrict__ woyp,
    const float* __restrict__ wozp, const float* __restrict__ ax, const float* __restrict__ ay,
    Eta e, float* __restrict__ pdf) {
    const int64_t tile = (int64_t)blockIdx.x * BLOCK * 4 * G;
    f4 x[G], y[G], z[G], ox[G], oy[G], oz[G], a[G], b[G];
    load_groups<G, BLOCK, true>(x, wix, tile, n);
    load_groups<G, BLOCK, true>(y, wiy, tile, n);
    load_groups<G, BLOCK, true>(z, wiz, tile, n);
    load_groups<G, BLOCK, true>(ox, woxp, tile, n);
    load_groups<G, BLOCK, true>(oy, woyp, tile, n);
    load_groups<G, BLOCK, true>(oz, wozp, tile, n);
    load_groups<G, BLOCK, true>(a, ax, tile, n);
    load_groups<G, BLOCK, true>(b, ay, tile, n);
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t i0 = group_start<G, BLOCK, true>(tile, g);
        if (i0 + 4 <= n) {
            f4 o;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                o[j] = dielectric_pdf_one(x[g][j], y[g][j], z[g][j], ox[g][j], oy[g][j], oz[g][j],
                                          a[g][j], b[g][j], e);
            store4_cached(pdf + i0, o);  // 4 B out per 32 B in
        } else {
            for (int64_t i = i0; i < n && i < i0 + 4; ++i)
                pdf[i] = dielectric_pdf_one(wix[i], wiy[i], wiz[i], woxp[i], woyp[i], wozp[i],
                                            ax[i], ay[i], e);
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_dielectric_pdf_scalar(
    int64_t n, const float* __restrict__ wix, const float* __restrict__ wiy,
    const float* __restrict__ wiz, const float* __restrict__ woxp, const float* __restrict__ woyp,
    const float* __restrict__ wozp, const float* __restrict__ ax, const float* __restrict__ ay,
    Eta e, float* __restrict__ pdf) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    pdf[i] = dielectric_pdf_one(wix[i], wiy[i], wiz[i], woxp[i], woyp[i], wozp[i], ax[i], ay[i], e);
}

int32_t make_eta(float eta, const char* who, Eta* out) {
    if (!(eta > 0.0f) || !(eta < INFINITY) || eta == 1.0f)
        return fail(CAPVNDF_ERR_BAD_ARG, "%s: eta must be finite, > 0 and != 1 (got %g)", who,
                    (double)eta);
    const double d = (double)eta;
    out->eta = eta;
    out->eta2 = (float)(d * d);
    out->eta2m1 = (float)(d * d - 1.0);
    out->ieta = (float)(1.0 / d);
    return CAPVNDF_OK;
}

}  // namespace
}  // namespace capvndf

using namespace capvndf;

extern "C" int32_t dielectric_sample(int64_t n, const float* wix, const float* wiy,
                                     const float* wiz, const float* ax, const float* ay,
                                     const float* u1, const float* u2, const float* u3, float eta,
                                     uint64_t seed, uint64_t index_base, float* wox, float* woy,
                                     float* woz, float* pdf, float* weight, void* stream) {
    if (n < 0) return fail(CAPVNDF_ERR_BAD_SIZE, "dielectric_sample: n = %lld < 0", (long long)n);
    Eta e;
    if (int32_t rc = make_eta(eta, "dielectric_sample", &e)) return rc;
    const bool eu = u1 != nullptr;
    if ((u2 != nullptr) != eu || (u3 != nullptr) != eu)
        return fail(CAPVNDF_ERR_NULL_PTR, "dielectric_sample: give all of u1, u2, u3 or none");
    if (n == 0) return CAPVNDF_OK;
    const void* req[] = {wix, wiy, wiz, ax, ay, wox, woy, woz, pdf, weight};
    const char* names[] = {"wix", "wiy", "wiz", "ax", "ay", "wox", "woy", "woz", "pdf", "weight"};
    bool vec = true;
    for (int i = 0; i < 10; ++i) {
        if (int32_t rc = check_array(req[i], names[i])) return rc;
        if (!aligned_to(req[i], 16)) vec = false;
    }
    if (eu) {
        const void* us[] = {u1, u2, u3};
        const char* un[] = {"u1", "u2", "u3"};
        for (int i = 0; i < 3; ++i) {
            if (int32_t rc = check_array(us[i], un[i])) return rc;
            if (!aligned_to(us[i], 16)) vec = false;
        }
    }
    const hipStream_t st = as_stream(stream);
    const uint32_t k0 = key_lo(seed), k1 = key_hi(seed);
    for (int64_t o = 0; o < n; o += kSliceElems) {
        const int64_t m = slice_len(n, o);
        const uint64_t ib = index_base + (uint64_t)o;
        const float *xi = wix + o, *yi = wiy + o, *zi = wiz + o, *axo = ax + o, *ayo = ay + o;
        const float *v1 = at(u1, o), *v2 = at(u2, o), *v3 = at(u3, o);
        float *xo = wox + o, *yo = woy + o, *zo = woz + o, *po = pdf + o, *wt = weight + o;
        if (vec) {
            const dim3 grid(tiles_for<kSampleGroups, kSampleBlock>(m)), block(kSampleBlock);
            if (eu)
                hipLaunchKernelGGL((k_dielectric_v4<kSampleGroups, kSampleBlock, true>), grid,
                                   block, 0, st, m, xi, yi, zi, axo, ayo, v1, v2, v3, e, ib, k0,
                                   k1, xo, yo, zo, po, wt);
            else
                hipLaunchKernelGGL((k_dielectric_v4<kSampleGroups, kSampleBlock, false>), grid,
                                   block, 0, st, m, xi, yi, zi, axo, ayo, v1, v2, v3, e, ib, k0,
                                   k1, xo, yo, zo, po, wt);
        } else {
            const dim3 grid(grid_for(m)), block(kBlock);
            if (eu)
                hipLaunchKernelGGL(k_dielectric_scalar<true>, grid, block, 0, st, m, xi, yi, zi,
                                   axo, ayo, v1, v2, v3, e, ib, k0, k1, xo, yo, zo, po, wt);
            else
                hipLaunchKernelGGL(k_dielectric_scalar<false>, grid, block, 0, st, m, xi, yi, zi,
                                   axo, ayo, v1, v2, v3, e, ib, k0, k1, xo, yo, zo, po, wt);
        }
        if (int32_t rc = check_launch("dielectric_sample launch")) return rc;
    }
    return CAPVNDF_OK;
}

extern "C" int32_t dielectric_pdf(int64_t n, const float* wix, const float* wiy, const float* wiz,
                                  const float* wox, const float* woy, const float* woz,
                                  const float* ax, const float* ay, float eta, float* pdf,
                                  void* stream) {
    if (n < 0) return fail(CAPVNDF_ERR_BAD_SIZE, "dielectric_pdf: n = %lld < 0", (long long)n);
    Eta e;
    if (int32_t rc = make_eta(eta, "dielectric_pdf", &e)) return rc;
    if (n == 0) return CAPVNDF_OK;
    const void* req[] = {wix, wiy, wiz, wox, woy, woz, ax, ay, pdf};
    const char* names[] = {"wix", "wiy", "wiz", "wox", "woy", "woz", "ax", "ay", "pdf"};
    bool vec = true;
    for (int i = 0; i < 9; ++i) {
        if (int32_t rc = check_array(req[i], names[i])) return rc;
        if (!aligned_to(req[i], 16)) vec = false;
    }
    const hipStream_t st = as_stream(stream);
    for (int64_t o = 0; o < n; o += kSliceElems) {
        const int64_t m = slice_len(n, o);
        if (vec)
            hipLaunchKernelGGL((k_dielectric_pdf_v4<kPdfGroups, kPdfBlock>),
                               dim3(tiles_for<kPdfGroups, kPdfBlock>(m)), dim3(kPdfBlock), 0, st,
                               m, wix + o, wiy + o, wiz + o, wox + o, woy + o, woz + o, ax + o,
                               ay + o, e, pdf + o);
        else
            hipLaunchKernelGGL(k_dielectric_pdf_scalar, dim3(grid_for(m)), dim3(kBlock), 0, st, m,
                               wix + o, wiy + o, wiz + o, wox + o, woy + o, woz + o, ax + o,
                               ay + o, e, pdf + o);
        if (int32_t rc = check_launch("dielectric_pdf launch")) return rc;
    }
    return CAPVNDF_OK;
}
